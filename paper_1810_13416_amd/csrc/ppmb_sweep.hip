// ppmb_sweep.hip -- the fused 1-D PPM + PPB pass for gfx950.
//
// One thread owns one pencil (a row of cells along the pass axis plus 4
// ghost cells per side, Sec. 4) and marches along it.  Each step loads one
// new cell and finishes the cell 4 behind it, so every stage of the pass
// (primitives, interface values, smoothness test and constraints, tracing,
// Riemann solve, fluxes, PPB slabs, update) works out of a short register
// window, the streaming form of the paper's pipelined pencil update
// (Sec. 4).  Lanes of a wave run across x, so for the y and z passes every
// load and store of a field is one coalesced 256-byte row.
#include "ppmb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>

namespace ppmb {

// Per-brick view handed to the pencil code: the brick's state, output and
// base fields, its dt and cell count.
template <typename T>
struct SweepArgs {
    const T *in;          // 15 fields, stride fs (pitched layout of Geom)
    T *out;
    const T *rho0;        // base state, working precision
    const T *p0;
    const double *dtp;    // this brick's dt
    unsigned long long *counters;   // limiter, unsmooth, riemann
    const double *r064;   // FP64 base state (for the fused CFL reduction)
    const double *p064;
    long fs;              // field stride (elements)
    int heat;             // 1: add the heating source after the update
    int cfl;              // 1: fold the written cells' signal speeds into the CFL slots
    T cthr;               // cells whose speed bound is below this need no FP64 speed
    const T *div;         // undivided velocity divergence (shock dissipation), same layout
    T dissk;              // shock dissipation coefficient
    const T *flat;        // flattening coefficients of this pass's input, same layout
    int skip;             // 1: solid cells hold the same values in both arenas; passes skip them
};

// Arguments of one pass launch over a batch of bricks.
template <typename T>
struct BatchArgs {
    const Brick *bricks;
    const BlockMap *map;
    const T *in;
    T *out;
    const T *base;
    const double *dt;
    unsigned long long *counters;
    const double *base64;
    unsigned long long *work;     // CFL slots, two per brick
    const unsigned long long *cband;   // per brick: FP64 bits of the band's lower edge, redo flag
    const T *div;                 // divergence field, one field per brick at boff / 2
    double dissk;                 // shock dissipation coefficient (kernels with DISS only)
    const T *flat;                // flattening field, one per brick at boff / 2 (FLAT only)
    int heat;
    int cfl;
    int skip;                     // solid cells are the same in both arenas: not written
    int chunk;                    // marching kernel: cells per wave along the pencil (0: all)
    int x_rows;                   // x pass: at least this many rows per wave
};

// A value that is the same on every lane, kept in scalar registers.
__device__ __forceinline__ float wave_uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double wave_uniform(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The band edge in the working precision, rounded down in FP32 so that no
// cell whose FP64 speed reaches the FP64 edge is judged below it.
__device__ __forceinline__ float band_edge(double v, float) { return __double2float_rd(v); }
__device__ __forceinline__ double band_edge(double v, double) { return v; }

template <typename T>
__device__ __forceinline__ SweepArgs<T> brick_args(const BatchArgs<T> &b, const Brick &B, int brick)
{
    // the same on every lane: kept in a scalar register
    const T thr = wave_uniform(b.cfl ? band_edge(__longlong_as_double((long long)b.cband[2 * brick]), T(0)) : T(0));
    return SweepArgs<T>{b.in + B.off, b.out + B.off, b.base + B.boff, b.base + B.boff + B.g.fs,
                        b.dt + B.dti, b.counters, b.base64 + B.boff, b.base64 + B.boff + B.g.fs,
                        B.g.fs, b.heat, b.cfl, thr, b.div ? b.div + B.boff / 2 : nullptr, T(b.dissk),
                        b.flat ? b.flat + B.boff / 2 : nullptr, b.skip};
}

// Global (x, y, z) order of a pass's (normal, t1, t2) components.
template <int AX, typename T>
__device__ __forceinline__ void to_global(T n, T t1, T t2, T &x, T &y, T &z)
{
    T c[3];
    c[AX] = n;
    c[(AX + 1) % 3] = t1;
    c[(AX + 2) % 3] = t2;
    x = c[0];
    y = c[1];
    z = c[2];
}

// One wave's share of the CFL reduction: maximum and non-physical flag over
// its lanes into the brick's slots (positive doubles order like their bits).
// A wave with no exact speed (no cell reached the band) adds nothing: the
// slot starts each pass at zero, so its maximum would change nothing.
__device__ __forceinline__ void cfl_commit(unsigned long long *work, int brick, double smax, bool bad)
{
    for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_down(smax, off));
    const unsigned long long bb = __ballot(bad);
    if ((threadIdx.x & 63) == 0) {
        if (smax > 0.0) atomicMax(&work[2 * brick], (unsigned long long)__double_as_longlong(smax));
        if (bb) atomicOr(&work[2 * brick + 1], 1ull);
    }
}

// One wave's event counts into its block's counter slot.
__device__ __forceinline__ void count_commit(unsigned long long *counters, unsigned c_lim, unsigned c_uns,
                                             unsigned c_rie)
{
    unsigned long long s0 = c_lim, s1 = c_uns, s2 = c_rie;
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_down(s0, off);
        s1 += __shfl_down(s1, off);
        s2 += __shfl_down(s2, off);
    }
    if ((threadIdx.x & 63) == 0) {
        unsigned long long *slot = counters + (blockIdx.x % kCntSlots) * kCntStride;
        if (s0) atomicAdd(&slot[0], s0);
        if (s1) atomicAdd(&slot[1], s1);
        if (s2) atomicAdd(&slot[2], s2);
    }
}

// Range-checked raw buffer access (gfx9 buffer resource, no stride): an
// element index at or past the resource's count reads zero and writes
// nothing, so stores are switched off per lane by their index, with no
// branch, and every address is a 32-bit lane offset from a wave-uniform base.
constexpr int kBufWord3 = 0x00020000;    // gfx9 raw buffer: 32-bit data format
constexpr unsigned kNoIdx = 1u << 28;    // past every resource made here
// A wave-uniform value passed through an empty asm: whatever is computed
// from it is recomputed at each use (a few scalar instructions) instead of
// being kept live in scalar registers across the loop, which would spill.
__device__ __forceinline__ long opaque_s(long v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// Gravity and heating parameters read from the brick table where they are
// used: scalar loads through a constant-memory pointer that the loop cannot
// hoist (waited for on the scalar counter), instead of values kept in
// vector registers across the loop, which at the register limit would be
// spilled; a spill reload is a vector memory load, and waiting for it
// waits for every load issued before it, the prefetches included.
using GeomC = const __attribute__((address_space(4))) Geom;
__device__ __forceinline__ GeomC *geom_c(const Geom *p)
{
    GeomC *q = (GeomC *)p;
    asm volatile("" : "+s"(q));
    return q;
}
__device__ __forceinline__ auto grav_c(GeomC *q, float) { return q->gcf; }
__device__ __forceinline__ auto grav_c(GeomC *q, double) { return q->gcd; }
__device__ __forceinline__ auto heat_c(GeomC *q, float) { return q->hcf; }
__device__ __forceinline__ auto heat_c(GeomC *q, double) { return q->hcd; }
template <typename T>
__device__ __forceinline__ T gravity_now(const Geom *p, int axis, T xd, T rt2)
{
    GeomC *q = geom_c(p);
    return gravity<T>(q->grav_kind, grav_c(q, T(0)), axis, xd, rt2);
}
template <typename T>
__device__ __forceinline__ T heating_now(const Geom *p, T z, T rt2)
{
    GeomC *q = geom_c(p);
    return heating<T>(q->heat_kind, heat_c(q, T(0)), z, rt2);
}

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const T *p, int count)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(p), 0, count * (int)sizeof(T), kBufWord3);
}
__device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, unsigned idx, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4u, 0, 0));
}
__device__ __forceinline__ double bld(__amdgpu_buffer_rsrc_t r, unsigned idx, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8u, 0, 0));
}
template <typename T>
__device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, unsigned idx)
{
    return bld(r, idx, T(0));
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned idx, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, idx * 4u, 0, 0);
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned idx, double v)
{
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, idx * 8u, 0, 0);
}

// A copy of v as a new value (an identity DPP move).  Loop-carried inputs
// loaded one step ahead are taken through it where they are consumed: the
// loaded registers then die there and the next step's loads can reuse them,
// instead of the compiler copying them at the loop latch, which would wait
// for the loads (and every store issued after them) at the end of each step.
template <typename T>
__device__ __forceinline__ T fresh(T v);
template <>
__device__ __forceinline__ float fresh(float v)
{
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, 0xE4, 0xf, 0xf, false));
}
template <>
__device__ __forceinline__ double fresh(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)b, (int)(unsigned)b, 0xE4, 0xf, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(b >> 32), (int)(unsigned)(b >> 32), 0xE4, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// pass-local order of the 10 fv coefficients and which flip at a wall
__host__ __device__ constexpr int mixed_of(int a, int b) { return FXY + (4 - a - b) % 3; }

template <int AX>
struct AxisInfo {
    static constexpr int t1 = (AX + 1) % 3, t2 = (AX + 2) % 3;
    static __device__ __forceinline__ int ppb(int q)
    {
        switch (q) {
        case 0: return F0;
        case 1: return FX + AX;
        case 2: return FXX + AX;
        case 3: return FX + t1;
        case 4: return mixed_of(AX, t1);
        case 5: return FX + t2;
        case 6: return mixed_of(AX, t2);
        case 7: return FXX + t1;
        case 8: return FXX + t2;
        default: return mixed_of(t1, t2);
        }
    }
    static __device__ __forceinline__ bool odd(int q) { return q == 1 || q == 4 || q == 6; }
};

// Rows of at most 32 pencils (along the lane axis of the marching kernel)
// are packed whole, 64 / n rows to a wave (a row split between two waves
// would have each of its loads touch the cache lines of two rows).
__host__ __device__ inline bool march_packed(const Geom &g, int axis)
{
    return g.n[axis == 0 ? 1 : 0] <= 32;
}
__host__ __device__ inline int march_rows(const Geom &g, int axis)
{
    return march_packed(g, axis) ? 64 / g.n[axis == 0 ? 1 : 0] : 1;
}

// Waves of the marching kernel per chunk of the pencils: packed rows, or
// columns of 64 pencils of one row.
__host__ __device__ inline long march_waves_per_chunk(const Geom &g, int axis)
{
    const int ca = axis == 0 ? 1 : 0, cb = 3 - axis - ca;
    const int R = march_rows(g, axis);
    return march_packed(g, axis) ? (g.n[cb] + R - 1) / R : (long)((g.n[ca] + 63) / 64) * g.n[cb];
}

// March one pencil; la / lb index it across the lane and block axes;
// gmem is the brick's grid in the brick table.
// Conserved perturbations (rho', m along the pass, the two transverse m,
// E') of a cell from its primitives q = (rho', u, v, w, p') and density rho.
template <typename T>
__device__ __forceinline__ void cons_of(const T *q, T rho, T rgm1, T *u)
{
    u[0] = q[0];
    u[1] = rho * q[1];
    u[2] = rho * q[2];
    u[3] = rho * q[3];
    u[4] = q[4] * rgm1 + T(0.5) * (u[1] * q[1] + u[2] * q[2] + u[3] * q[3]);
}

template <typename T, int AX, bool DISS, bool FLAT>
__device__ void march(const Geom &g, const Geom *gmem, const SweepArgs<T> &a, int la0, int lane, int lb,
                      int clo, int chi, unsigned &c_lim, unsigned &c_uns, unsigned &c_rie, double &cmax,
                      bool &cbad)
{
    using AI = AxisInfo<AX>;
    const int n = g.n[AX];
    const int ca = (AX == 0) ? 1 : 0;
    const int cb = 3 - AX - ca;
    // The wave's pencils.  Rows (along cb) of g.n[ca] pencils: a row of
    // more than 32 pencils gives waves the 64 from la0 of row lb; shorter
    // rows are packed whole, lane after lane, rows lb .. lb + 64 / n - 1
    // (la0 = 0).  Lanes past the last pencil march a copy of it and store
    // nothing.
    const int na = g.n[ca], nrow = g.n[cb];
    const bool packed = march_packed(g, AX);
    const int last = packed ? min(march_rows(g, AX), nrow - lb) * na - 1 : 0;
    int lld, lrow;
    bool valid;
    if (packed) {
        valid = lane <= last;
        const int pe = valid ? lane : last;
        lrow = pe / na;
        lld = pe - lrow * na;
    } else {
        const int cnt = min(64, na - la0);
        valid = lane < cnt;
        lld = valid ? lane : cnt - 1;
        lrow = 0;
    }
    const int la = la0 + lld;
    int ijk0[3];
    ijk0[ca] = la; ijk0[cb] = lb + lrow; ijk0[AX] = 0;
    const long stride[3] = { 1, (long)g.px, g.plane };
    const long sAX = stride[AX];
    // element index of this lane from the wave's first row start (stride 1
    // for the y and z passes, nx for the x pass, rows stride[cb] apart), and
    // the element count the wave's pencils span (the index grows with the
    // pencil number, so the last lane's is the largest)
    const unsigned lix = (unsigned)(lld * stride[ca] + lrow * stride[cb]);
    const unsigned lst = valid ? lix : kNoIdx;
    const int rcnt = (int)__builtin_amdgcn_readlane((int)lix, 63) + 1;
    // wave-uniform offset of row lb's pencil la0
    const long ubase = (long)la0 * stride[ca] + (long)lb * stride[cb];
    const double xt[3] = { centre(g, 0, ijk0[0]), centre(g, 1, ijk0[1]), centre(g, 2, ijk0[2]) };
    // transverse part of |x|^2 and the fluid interval of this pencil
    const T xt1 = T(xt[AI::t1]), xt2 = T(xt[AI::t2]);
    const T rtt = xt1 * xt1 + xt2 * xt2;
    // z of the pencil for the heating when z is transverse: the coordinate of
    // the wave's row (lb), the same on every lane unless rows are packed
    // (then rebuilt from the lane where it is used)
    const T zt = AX == 2 ? T(0) : wave_uniform(T(xt[2]));
    int flo, fhi;
    fluid_interval(g, AX, xt, flo, fhi);
    const T ox = T(g.origin[AX]), dxT = T(g.dx);
    // The cells the wave updates: [wlo, whi], its chunk [clo, chi] of the
    // pencils, narrowed when solid cells are skipped (they keep their
    // values, which both arenas hold alike) to the union of the pencils'
    // fluid cells in the chunk.  The march reads 4 cells beyond it on
    // either side (real cells, solid ones included, or ghosts through the
    // boundary conditions) and writes only inside it.
    int wlo = clo, whi = chi;
    if (a.skip) {
        const int fl = max(flo, clo), fh = min(fhi, chi);
        int l = fl <= fh ? fl : n, h = fl <= fh ? fh : -1;
        for (int off = 1; off < 64; off <<= 1) {
            l = min(l, __shfl_xor(l, off));
            h = max(h, __shfl_xor(h, off));
        }
        wlo = __builtin_amdgcn_readfirstlane(l);
        whi = __builtin_amdgcn_readfirstlane(h);
        if (wlo > whi) return;             // every pencil of the wave is solid
    }
    const int k0 = wlo - NG;               // first cell loaded

    const double dt64 = *a.dtp;
    const T dt = T(dt64), nu = T(dt64 / g.dx), hdt = T(0.5 * dt64), rdx = T(1.0 / g.dx);
    const T gam = T(g.gamma), gm1 = T(g.gamma - 1.0), gfac = T(g.gamma / (g.gamma - 1.0));
    const T rgm1 = T(1.0 / (g.gamma - 1.0));
    const int bc = g.bc[AX];
    const T *in = a.in;
    const long nc = a.fs;
    // field q of the 64-lane row at pencil index s (in / out / base)
    const T *inb = in + ubase;
    T *outb = a.out + ubase;
    auto rin = [&](int q, int s) { return rsrc(inb + (opaque_s(nc) * q + s * sAX), rcnt); };
    auto rout = [&](int q, int s) { return rsrc(outb + (opaque_s(nc) * q + s * sAX), rcnt); };

    // --- register window ---------------------------------------------
    T q[5][5];            // primitives rho', u, v, w, p' of cells k-4..k
    T rr[3], cr[3];       // rho, c of cells k-2..k
    T irr[3], icr[3];     // their reciprocals
    T b0[4], b1[4];       // base rho0, p0 of cells k-3..k
    T gr[4];              // gravity along the pass, cells k-3..k
    bool sol[5];          // solid flags of cells k-4..k
    T qf[2][5], r0f[2], p0f[2];   // faces (k-3)+1/2 and (k-2)+1/2
    T sm[3][5];           // limited slopes of cells k-3..k-1
    T d2[3][5];           // second differences of cells k-3..k-1
    T flm[2][5];          // limited-slope face values at (k-3)+1/2, (k-2)+1/2
    St<T> TLp;            // right-face state of cell k-3
    T Fp[5];              // fluxes at face (k-4)+1/2
    T sg1 = T(0), sg2 = T(0);     // sigma at faces (k-4)+1/2, (k-5)+1/2
    T pq[10], pqp[10];    // fv coefficients of cells k-3 (this step) and k-4 (limited)
    T pqr1 = T(0), pqr2 = T(0);   // cell k-4's slope and curvature before limiting
    T Lp = T(1);          // Lagrangian length of cell k-4
    T Gp[10];             // slab at face (k-5)+1/2
    T dvp = T(0), dvc = T(0);     // shock dissipation: divergence of cells k-3, k-2
    T fk = T(0);                  // flattening coefficient of cell k-2
    for (int v = 0; v < 5; ++v) Fp[v] = T(0);
    for (int v = 0; v < 10; ++v) { pq[v] = T(0); pqp[v] = T(0); Gp[v] = T(0); }
    TLp = St<T>{T(0), T(0), T(0), T(0), T(0)};
    for (int c = 0; c < 4; ++c) { gr[c] = T(0); b0[c] = T(0); b1[c] = T(0); }
    for (int c = 0; c < 5; ++c) sol[c] = false;

    // Inputs of the next cell, loaded one step ahead so that their latency
    // hides behind the current step's arithmetic.
    T nx_rp, nx_mn, nx_m1, nx_m2, nx_ep, nx_r0, nx_pb;
    int nx_s, nx_fl;
    auto load_next = [&](int k) {
        int fl = 1;
        int s = k;
        if (k < 0 || k >= n) s = bc_source(k, n, bc, fl);
        nx_rp = bld<T>(rin(RHO, s), lix);
        nx_mn = bld<T>(rin(MX + AX, s), lix);
        nx_m1 = bld<T>(rin(MX + AI::t1, s), lix);
        nx_m2 = bld<T>(rin(MX + AI::t2, s), lix);
        nx_ep = bld<T>(rin(EN, s), lix);
        nx_r0 = bld<T>(rsrc(a.rho0 + ubase + s * sAX, rcnt), lix);
        nx_pb = bld<T>(rsrc(a.p0 + ubase + s * sAX, rcnt), lix);
        nx_s = s;
        nx_fl = fl;
    };
    load_next(k0);
    // settle the first loads here, so that the loop's own wait for the next
    // cell's inputs only counts memory operations issued after them
    __builtin_amdgcn_s_waitcnt(0);
    {
        // The window starts filled with the first cell's state, so that the
        // first steps, whose results are not stored (an update reads only
        // cells within 4 of its own), compute on physical values.
        const T flT = T(nx_fl);
        const T rho = nx_r0 + nx_rp, ir = trcp(rho);
        const T mn = flT * nx_mn;
        const T u = mn * ir, v = nx_m1 * ir, w = nx_m2 * ir;
        const T pp = gm1 * (nx_ep - T(0.5) * (mn * u + nx_m1 * v + nx_m2 * w));
        T c, ic;
        sound(gam * (nx_pb + pp) * ir, c, ic);
        const T pv[5] = { nx_rp, u, v, w, pp };
#pragma unroll
        for (int vv = 0; vv < 5; ++vv) {
#pragma unroll
            for (int r = 0; r < 5; ++r) q[r][vv] = pv[vv];
#pragma unroll
            for (int r = 0; r < 2; ++r) { qf[r][vv] = pv[vv]; flm[r][vv] = pv[vv]; }
#pragma unroll
            for (int r = 0; r < 3; ++r) { sm[r][vv] = T(0); d2[r][vv] = T(0); }
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) { rr[r] = rho; cr[r] = c; irr[r] = ir; icr[r] = ic; }
#pragma unroll
        for (int r = 0; r < 4; ++r) { b0[r] = nx_r0; b1[r] = nx_pb; }
#pragma unroll
        for (int r = 0; r < 2; ++r) { r0f[r] = nx_r0; p0f[r] = nx_pb; }
        TLp = St<T>{nx_rp, u, v, w, pp};
    }

    // One step of the march.  Every step runs every stage with the same
    // arithmetic (so a cell's result does not depend on where its wave's
    // range begins or ends); only the stores and the event counts are
    // switched off outside the range, by index, so that every memory
    // operation is issued on every step and the compiler's waits count
    // exactly the operations issued after the one waited for.
    auto step = [&](const int k) {
        // ---- (1) cell k from the prefetched inputs (base added back, Sec. 1);
        //          loads of cell k+1 and of the conserved fields of cell k-3
        //          (cache hits, for its update) are issued first
        const int s = nx_s;
        const T flT = T(nx_fl);
        const T rp = fresh(nx_rp), mn = flT * nx_mn, m1 = fresh(nx_m1), m2 = fresh(nx_m2), ep = fresh(nx_ep);
        const T r0 = fresh(nx_r0), pb = fresh(nx_pb);
        const int cu_ = k - 3;
        const bool upd = cu_ >= wlo && cu_ <= whi;
        // cell k-3 (through the boundary conditions outside the pencil,
        // where the wall flip of the normal momentum is applied below):
        // its conserved fields for its update, its fv coefficients (donors
        // -1..n) for the PPB stage, loaded raw; no arithmetic waits on these
        // loads before they are used
        int pq_fl = 1;
        int s3 = cu_;
        if (s3 < 0 || s3 >= n) s3 = bc_source(cu_, n, bc, pq_fl);
        const unsigned st3 = upd ? lst : kNoIdx;
        T cu3[5];
        cu3[0] = bld<T>(rin(RHO, s3), lix);
        cu3[1] = bld<T>(rin(MX + AX, s3), lix);
        cu3[2] = bld<T>(rin(MX + AI::t1, s3), lix);
        cu3[3] = bld<T>(rin(MX + AI::t2, s3), lix);
        cu3[4] = bld<T>(rin(EN, s3), lix);
        if constexpr (DISS || FLAT) {
            // divergence of cell k-2 for the face (k-3)+1/2 (that of cell
            // k-3 is carried from the previous step) and the flattening
            // coefficient of cell k-2 for its parabola
            int s2 = k - 2, f2;
            if (s2 < 0 || s2 >= n) s2 = bc_source(s2, n, bc, f2);
            if constexpr (DISS) {
                dvp = dvc;
                dvc = bld<T>(rsrc(a.div + ubase + s2 * sAX, rcnt), lix);
            }
            if constexpr (FLAT) fk = bld<T>(rsrc(a.flat + ubase + s2 * sAX, rcnt), lix);
        }
        {
            T xd = ox + (T(s) + T(0.5)) * dxT;
            T gv = flT * gravity_now<T>(gmem, AX, xd, rtt + xd * xd);
            bool so = s < flo || s > fhi;
            T rho = r0 + rp;
            T ir = trcp(rho);
            T u = mn * ir, v = m1 * ir, w = m2 * ir;
            T pp = gm1 * (ep - T(0.5) * (mn * u + m1 * v + m2 * w));
            T c, ic;
            sound(gam * (pb + pp) * ir, c, ic);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int vv = 0; vv < 5; ++vv) q[r][vv] = q[r + 1][vv];
            q[4][0] = rp; q[4][1] = u; q[4][2] = v; q[4][3] = w; q[4][4] = pp;
            rr[0] = rr[1]; rr[1] = rr[2]; rr[2] = rho;
            cr[0] = cr[1]; cr[1] = cr[2]; cr[2] = c;
            irr[0] = irr[1]; irr[1] = irr[2]; irr[2] = ir;
            icr[0] = icr[1]; icr[1] = icr[2]; icr[2] = ic;
#pragma unroll
            for (int r = 0; r < 3; ++r) { b0[r] = b0[r + 1]; b1[r] = b1[r + 1]; gr[r] = gr[r + 1]; }
#pragma unroll
            for (int r = 0; r < 4; ++r) sol[r] = sol[r + 1];
            b0[3] = r0; b1[3] = pb; gr[3] = gv; sol[4] = so;
        }
        // the inputs of cell k are consumed: their registers take the loads
        // of cell k+1 (past the end this reads a valid ghost source, unused).
        // The barrier keeps the scheduler from hoisting these loads above
        // the last use of the old values, which would force a register copy
        // (and a wait on the loads) at the end of every step.
        __builtin_amdgcn_sched_barrier(0);
        load_next(k + 1);
#pragma unroll
        for (int v = 0; v < 10; ++v) pq[v] = bld<T>(rin(AI::ppb(v), s3), lix);
        // ---- (2) interface values at face (k-2)+1/2 (cells k-3..k)
        {
#pragma unroll
            for (int vv = 0; vv < 5; ++vv) { qf[0][vv] = qf[1][vv]; qf[1][vv] = face4(q[1][vv], q[2][vv], q[3][vv], q[4][vv]); }
            r0f[0] = r0f[1]; r0f[1] = face4(b0[0], b0[1], b0[2], b0[3]);
            p0f[0] = p0f[1]; p0f[1] = face4(b1[0], b1[1], b1[2], b1[3]);
        }
        // ---- (3) limited slope and second difference of cell k-1; the
        //          limited-slope face value at (k-2)+1/2
        {
#pragma unroll
            for (int vv = 0; vv < 5; ++vv) {
                sm[0][vv] = sm[1][vv]; sm[1][vv] = sm[2][vv];
                sm[2][vv] = limited_slope(q[2][vv], q[3][vv], q[4][vv]);
                d2[0][vv] = d2[1][vv]; d2[1][vv] = d2[2][vv];
                d2[2][vv] = (q[2][vv] + q[4][vv]) - T(2) * q[3][vv];
                flm[0][vv] = flm[1][vv];
                flm[1][vv] = face_limited(q[2][vv], q[3][vv], sm[1][vv], sm[2][vv]);
            }
        }
        // ---- (4) parabolas of cell k-2, constrained only where the 5-cell
        //          window is not smooth (Sec. 1), blended over the graded
        //          band; tracing (CW84 Sec. 3)
        St<T> TL, TR;
        {
            // unsmooth pairs are counted in the fluid cells the wave updates
            const bool interior = (k - 2 >= wlo) && (k - 2 <= whi) && !sol[2];
            T qL[5], qR[5], dq[5], q6[5];
#pragma unroll
            for (int vv = 0; vv < 5; ++vv) {
                T l, r;
                bool con = parabola(g.smooth_detect, q[2][vv], qf[0][vv], qf[1][vv], flm[0][vv], flm[1][vv],
                                    d2[0][vv], d2[1][vv], d2[2][vv], l, r);
                if (con && interior && valid) ++c_uns;
                if constexpr (FLAT) {
                    // flattening toward the cell average near strong shocks
                    l = fk * q[2][vv] + (T(1) - fk) * l;
                    r = fk * q[2][vv] + (T(1) - fk) * r;
                }
                qL[vv] = l; qR[vv] = r;
                dq[vv] = r - l;
                q6[vv] = T(6) * (q[2][vv] - T(0.5) * (l + r));
            }
            trace_cell(qL, qR, dq, q6, rr[0], irr[0], cr[0], icr[0], q[2][1], q[2][0], gr[1], r0f[0], r0f[1],
                       p0f[0], p0f[1], nu, hdt, rdx, TL, TR);
        }
        // ---- (5) Riemann problem and fluxes at face (k-3)+1/2
        T F[5];
        T sg;
        {
            bool rie = face_flux<T>(TLp, TR, sol[1], sol[2], r0f[0], p0f[0], gam, gfac, nu, F, sg);
            if (rie && (k - 3 >= wlo - 1) && (k - 3 <= whi) && valid) ++c_rie;
            if constexpr (DISS) {
                // shock dissipation across a face between fluid cells: the
                // conserved fields of cell k-3 as loaded for its update, and
                // those of cell k-2 rebuilt from its primitives
                const T nv = (sol[1] || sol[2]) ? T(0) : a.dissk * tmax(T(0), T(-0.5) * (dvp + dvc));
                T ub[5];
                cons_of(q[2], rr[0], rgm1, ub);
                if (pq_fl < 0) cu3[1] = -cu3[1];     // seen through a reflecting wall
#pragma unroll
                for (int vv = 0; vv < 5; ++vv) F[vv] = F[vv] + nv * (cu3[vv] - ub[vv]);
            }
        }
        TLp = TL;
        // ---- (6) conservative update of cell k-3 and heating; written now
        {
            // (outside the pencil the update is not stored; DISS has flipped
            // the ghost's normal momentum already)
            if constexpr (!DISS) {
                if (pq_fl < 0) cu3[1] = -cu3[1];
            }
            T hn[5];
            hydro_update(cu3, Fp, F, nu, dt, gr[0], hn);
            if (a.heat) {
                T xd = ox + (T(cu_) + T(0.5)) * dxT;
                T zc = AX == 2 ? xd : zt;
                if (AX != 2 && packed) {
                    // the lane id from the exec mask, so that no register
                    // holds it through the march
                    const int ln = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
                    zc = T(centre(g, 2, lb + min(ln, last) / na));
                }
                hn[4] = hn[4] + heating_now<T>(gmem, zc, rtt + xd * xd) * dt;
            }
#pragma unroll
            for (int vv = 0; vv < 5; ++vv) hn[vv] = sol[1] ? cu3[vv] : hn[vv];
            bst(rout(RHO, s3), st3, hn[0]);
            bst(rout(MX + AX, s3), st3, hn[1]);
            bst(rout(MX + AI::t1, s3), st3, hn[2]);
            bst(rout(MX + AI::t2, s3), st3, hn[3]);
            bst(rout(EN, s3), st3, hn[4]);
            // the next step's CFL reduction from the values just written:
            // the exact FP64 speed only where the bound reaches the band
            // below the last maximum (in few waves), with its FP64 base
            if (a.cfl) {
                const bool need = upd && valid && !sol[1] &&
                                  speed_may_reach(b0[0], b1[0], hn[0], hn[1], hn[2], hn[3], hn[4], gam, gm1, a.cthr);
                if (__ballot(need)) {
                    const unsigned ic = need ? lix : kNoIdx;
                    const double br0 = bld<double>(rsrc(a.r064 + ubase + s3 * sAX, rcnt), ic);
                    const double bp0 = bld<double>(rsrc(a.p064 + ubase + s3 * sAX, rcnt), ic);
                    if (need) {
                        double mx, my, mz;
                        to_global<AX, double>(hn[1], hn[2], hn[3], mx, my, mz);
                        bool bd;
                        const double sp = cell_speed(br0, bp0, (double)hn[0], mx, my, mz, (double)hn[4], g.gamma, bd);
                        if (bd) cbad = true;
                        else cmax = fmax(cmax, sp);
                    }
                }
            }
        }
        // ---- (7) PPB: donor k-3, slab at face (k-4)+1/2, update cell k-4
        {
            if (pq_fl < 0) {
#pragma unroll
                for (int v = 0; v < 10; ++v) pq[v] = AI::odd(v) ? -pq[v] : pq[v];
            }
            T Ld = T(1) + (sg - sg1);
            T l1 = pq[1], l2 = pq[2];
            bool hit = fv_limit(pq[0], l1, l2);
            if (hit && upd && !sol[1] && valid) ++c_lim;
            T pql[10];
#pragma unroll
            for (int v = 0; v < 10; ++v) pql[v] = pq[v];
            pql[1] = l1; pql[2] = l2;
            T G[10];
            {
                // donor: cell k-4 when the face velocity is positive, else
                // cell k-3 seen mirrored (odd-in-s coefficients flipped); a
                // zero velocity gives a zero slab
                const bool pos = sg1 > T(0);
                T dn[10];
#pragma unroll
                for (int v = 0; v < 10; ++v) {
                    const T f = (v == 1 || v == 4 || v == 6) ? -pql[v] : pql[v];
                    dn[v] = pos ? pqp[v] : f;
                }
                slab(dn, sg1, pos ? Lp : Ld, G);
                const int cw = k - 4;
                const bool wr = cw >= wlo && cw <= whi;
                const int cwc = wr ? cw : wlo;
                const unsigned stw = wr ? lst : kNoIdx;
                T o[10];
                ppb_update(pqp, sg1 - sg2, T(0.5) * (sg2 + sg1), Gp, G, o);
                // a solid cell keeps its coefficients as they came in
#pragma unroll
                for (int v = 0; v < 10; ++v)
                    o[v] = sol[0] ? (v == 1 ? pqr1 : (v == 2 ? pqr2 : pqp[v])) : o[v];
#pragma unroll
                for (int v = 0; v < 10; ++v) bst(rout(AI::ppb(v), cwc), stw, o[v]);
#pragma unroll
                for (int v = 0; v < 10; ++v) Gp[v] = G[v];
            }
#pragma unroll
            for (int v = 0; v < 10; ++v) pqp[v] = pql[v];
            pqr1 = pq[1];
            pqr2 = pq[2];
            Lp = Ld;
        }
        sg2 = sg1; sg1 = sg;
#pragma unroll
        for (int vv = 0; vv < 5; ++vv) Fp[vv] = F[vv];
    };
    for (int k = k0; k <= whi + NG; ++k) step(k);
}

// Marching kernel: each wave covers 64 pencils (lanes across x for the y
// and z passes, across y for the x pass); a block holds blockDim/64 waves
// on consecutive rows of the other transverse axis.
// FP32: at most 256 VGPRs, two waves per SIMD; FP64 needs the full file.


// Waves of the marching kernel along a pencil of n cells: chunks of
// `chunk` cells (0: one wave for the whole pencil).  Each wave marches its
// chunk plus 4 cells either side.
__host__ __device__ inline int march_chunks(int n, int chunk)
{
    return chunk > 0 ? (n + chunk - 1) / chunk : 1;
}

// Wave wv of the `waves` waves of marching block m.
template <typename T, int AX, bool DISS, bool FLAT>
__device__ __forceinline__ void march_wave(const BatchArgs<T> &b, const BlockMap m, int wv, int waves)
{
    const Brick &B = b.bricks[m.brick];
    const Geom g = B.g;
    const SweepArgs<T> a = brick_args(b, B, m.brick);
    const int ca = (AX == 0) ? 1 : 0;
    const int cb = 3 - AX - ca;
    const int nblk_a = (g.n[ca] + 63) / 64;
    // block = (chunk along the pencils, its waves); a wave = 64 packed
    // pencils, or a column of 64 pencils of one row
    const int nchk = march_chunks(g.n[AX], b.chunk);
    const int ck = m.local % nchk, rest = m.local / nchk;
    const long wq = (long)rest * waves + wv;
    int la0, lb;
    if (march_packed(g, AX)) {
        la0 = 0;
        lb = (int)(wq * march_rows(g, AX));
    } else {
        la0 = (int)(wq % nblk_a) * 64;
        lb = (int)(wq / nblk_a);
    }
    const int clen = b.chunk > 0 ? b.chunk : g.n[AX];
    const int clo = ck * clen, chi = min(clo + clen, g.n[AX]) - 1;
    unsigned c_lim = 0, c_uns = 0, c_rie = 0;          // per lane; widened below
    double cmax = 0.0;
    bool cbad = false;
    if (lb < g.n[cb])
        march<T, AX, DISS, FLAT>(g, &B.g, a, la0, (int)(threadIdx.x & 63), lb, clo, chi, c_lim, c_uns, c_rie,
                                 cmax, cbad);
    if (b.cfl) cfl_commit(b.work, m.brick, cmax, cbad);
    count_commit(a.counters, c_lim, c_uns, c_rie);
}

template <typename T, int AX, bool DISS, bool FLAT>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1)
void sweep_kernel(BatchArgs<T> b)
{
    march_wave<T, AX, DISS, FLAT>(b, b.map[blockIdx.x], __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)),
                                  (int)(blockDim.x >> 6));
}

// ---------------------------------------------------------------------
// x pass with lanes along x.  Marching along x with lanes across y would
// make every load touch 64 separate cache lines; instead one wave holds 64
// consecutive cells of one x-pencil (cells x0-4 .. x0+59), every load and
// store of a field is one coalesced 256-byte row, neighbours come from
// whole-wave shifts, and the wave finishes the middle 56 cells, whose
// 4-cell dependency cone (Sec. 4) lies inside the wave; then it moves 56
// cells on along the same row.
// ---------------------------------------------------------------------

constexpr int kXOut = 56;
constexpr int kXItems = 8;     // (row, segment) items per wave, at least

// Items per wave: whole rows, at least kXItems items and min_rows rows.
__host__ __device__ __forceinline__ int x_run(int nseg, int min_rows)
{
    int rows = kXItems / nseg;
    rows = rows > min_rows ? rows : min_rows;
    return (rows > 1 ? rows : 1) * nseg;
}

// Neighbour values inside the wave by DPP whole-wave shifts (wave_shr:1,
// wave_shl:1): a VALU move, no LDS round trip.  The lane at the wave's edge
// reads zero (bound_ctrl): its results are halo, outside every owned
// cell's dependency cone, and with no old value to keep the shift needs no
// register copy and can fold into the instruction that uses it.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_v(float v)
{
    return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_v(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)dpp_i<CTRL>((int)(unsigned)b);
    const unsigned hi = (unsigned)dpp_i<CTRL>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
constexpr int kWaveShr1 = 0x138;   // lane l reads lane l - 1
constexpr int kWaveShl1 = 0x130;   // lane l reads lane l + 1

// value of the cell on the left (lane - 1) and on the right (lane + 1)
template <typename T>
__device__ __forceinline__ T from_left(T v) { return dpp_v<kWaveShr1>(v); }
template <typename T>
__device__ __forceinline__ T from_right(T v) { return dpp_v<kWaveShl1>(v); }
__device__ __forceinline__ int from_right_i(int v) { return dpp_i<kWaveShl1>(v); }

template <typename T>
__device__ __forceinline__ St<T> from_right(const St<T> &v)
{
    return St<T>{from_right(v.r), from_right(v.u), from_right(v.v), from_right(v.w), from_right(v.p)};
}

// Inputs of one lane for one segment: its cell's conserved fields, fv
// coefficients (pass order, odd ones flipped through a wall) and base.
template <typename T>
struct XIn {
    T cu[5];
    T pq[10];
    T r0, pb;
    T dv;             // divergence (shock dissipation only)
    double fr0, fp0;  // FP64 base (flattening only)
    int s, fl;
};

template <typename T, bool DISS, bool FLAT>
__device__ __forceinline__ void x_load(const T *in, const T *rho0, const T *p0, const T *div, const double *r064,
                                       const double *p064, long nc, long row,
                                       int nx, int bc, int i, XIn<T> &o)
{
    using AI = AxisInfo<0>;
    int fl = 1;
    int s = i;
    if (i < 0 || i >= nx) s = bc_source(i, nx, bc, fl);
    o.s = s;
    o.fl = fl;
    const T *inr = in + row;
    auto fld = [&](int q) { return rsrc(inr + opaque_s(nc) * q, nx); };
    o.cu[0] = bld<T>(fld(RHO), s);
    o.cu[1] = bld<T>(fld(MX), s);
    o.cu[2] = bld<T>(fld(MY), s);
    o.cu[3] = bld<T>(fld(MZ), s);
    o.cu[4] = bld<T>(fld(EN), s);
#pragma unroll
    for (int v = 0; v < 10; ++v) o.pq[v] = bld<T>(fld(AI::ppb(v)), s);
    o.r0 = bld<T>(rsrc(rho0 + row, nx), s);
    o.pb = bld<T>(rsrc(p0 + row, nx), s);
    if constexpr (DISS) o.dv = bld<T>(rsrc(div + row, nx), s);
    if constexpr (FLAT) {
        if constexpr (sizeof(T) == 8) {
            o.fr0 = o.r0;
            o.fp0 = o.pb;
        } else {
            o.fr0 = bld<double>(rsrc(r064 + row, nx), s);
            o.fp0 = bld<double>(rsrc(p064 + row, nx), s);
        }
    }
}

// One wave walks whole x-rows, 56-cell segment by segment, at least
// kXItems segments (several rows when they are short, as in small bricks),
// so that each wave has enough work; the loads of the next segment (of the
// same or the next row) are issued before the current one is computed, so
// their latency hides behind the arithmetic.
// Wave wv (counted over the brick's x-pass waves) of x block m.
template <typename T, bool DISS, bool FLAT>
__device__ __forceinline__ void x_wave(const BatchArgs<T> &b, const BlockMap m, const int wv)
{
    using AI = AxisInfo<0>;
    const Brick &B = b.bricks[m.brick];
    const Geom g = B.g;
    const SweepArgs<T> a = brick_args(b, B, m.brick);
    const int lane = threadIdx.x & 63;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    // this wave's run of items: item = (x-row, segment), rows in storage
    // order, segments along the row
    const int nseg = (nx + kXOut - 1) / kXOut;
    const int items = ny * nz * nseg;
    const int run = x_run(nseg, b.x_rows);
    const int it0 = wv * run;                          // whole rows: it0 is a row start
    if (it0 >= items) return;                          // whole waves only
    const int it1 = min(it0 + run, items);
    const long nc = a.fs;
    const double dt64 = *a.dtp;
    const T dt = T(dt64), nu = T(dt64 / g.dx), hdt = T(0.5 * dt64), rdx = T(1.0 / g.dx);
    const T gam = T(g.gamma), gm1 = T(g.gamma - 1.0), gfac = T(g.gamma / (g.gamma - 1.0));
    const T ox = T(g.origin[0]), dxT = T(g.dx);
    const int bc = g.bc[0];
    unsigned c_lim = 0, c_uns = 0, c_rie = 0;          // per lane; widened below
    double cmax = 0.0;                                 // fused CFL reduction
    bool cbad = false;

    // The work on row r: ns segments of 56 output cells from cell x0.
    // With solid cells skipped (both arenas hold them alike) the segments
    // start at the row's first fluid cell and end at or past its last (none
    // for an all-solid row); else they tile the whole row from 0.
    auto row_work = [&](int r, int &x0, int &ns) {
        x0 = 0;
        ns = nseg;
        if (!a.skip || !g.sphere) return;
        const double xt[3] = { 0.0, centre(g, 1, r % ny), centre(g, 2, r / ny) };
        int flo, fhi;
        fluid_interval(g, 0, xt, flo, fhi);
        x0 = __builtin_amdgcn_readfirstlane(flo);
        ns = __builtin_amdgcn_readfirstlane(flo <= fhi ? (fhi - flo) / kXOut + 1 : 0);
    };
    // the first row from r on (below rend) with work, and that work
    const int rend = (it1 + nseg - 1) / nseg;
    auto next_row = [&](int r, int &x0, int &ns) {
        for (; r < rend; ++r) {
            row_work(r, x0, ns);
            if (ns > 0) break;
        }
        return r;
    };

    int rowi, rx0, rns;
    rowi = next_row(it0 / nseg, rx0, rns);
    XIn<T> cur;
    if (rowi < rend)
        x_load<T, DISS, FLAT>(a.in, a.rho0, a.p0, a.div, a.r064, a.p064, nc, (long)rowi * g.px, nx, bc, rx0 - NG + lane,
                              cur);
    // settle the first loads, so that the loop's waits count only the
    // memory operations of the loop itself
    __builtin_amdgcn_s_waitcnt(0);
    while (rowi < rend) {
      const int y = rowi % ny, z = rowi / ny;
      const long row = (long)rowi * g.px;
      const double yc = centre(g, 1, y), zc = centre(g, 2, z);
      const T xt1 = T(yc), xt2 = T(zc);
      const T rtt = xt1 * xt1 + xt2 * xt2;
      // the row after this one with work (its loads start at this row's
      // last segment)
      int nx0 = 0, nns = 0;
      const int nrow = next_row(rowi + 1, nx0, nns);
      for (int seg = 0; seg < rns; ++seg) {
        const int i = rx0 + seg * kXOut - NG + lane;   // this lane's cell along x

        // (1) this lane's cell: its inputs are taken over as new values,
        //     then the next segment's loads go into the same registers
        //     (past the row's end they read valid ghost sources, unused)
        const int s = cur.s;
        const T fl = T(cur.fl);
        T cu[5], pq[10];
        cu[0] = fresh(cur.cu[0]);
        cu[1] = fl * cur.cu[1];
        cu[2] = fresh(cur.cu[2]);
        cu[3] = fresh(cur.cu[3]);
        cu[4] = fresh(cur.cu[4]);
#pragma unroll
        for (int v = 0; v < 10; ++v) pq[v] = AI::odd(v) ? fl * cur.pq[v] : fresh(cur.pq[v]);
        const T r0 = fresh(cur.r0), pb = fresh(cur.pb);
        T dv = T(0);
        if constexpr (DISS) dv = fresh(cur.dv);
        double fr0 = 0.0, fp0 = 0.0;
        if constexpr (FLAT) {
            fr0 = fresh(cur.fr0);
            fp0 = fresh(cur.fp0);
        }
        __builtin_amdgcn_sched_barrier(0);
        {
            // the next item: this row's next segment, else the next row's
            // first; past the run this one again (loaded, unused)
            const bool more = seg + 1 < rns;
            const int ni = more ? rx0 + (seg + 1) * kXOut : (nrow < rend ? nx0 : rx0 + seg * kXOut);
            const long nr = more ? row : (nrow < rend ? (long)nrow * g.px : row);
            x_load<T, DISS, FLAT>(a.in, a.rho0, a.p0, a.div, a.r064, a.p064, nc, nr, nx, bc, ni - NG + lane, cur);
        }
        const T xd = ox + (T(s) + T(0.5)) * dxT;
        const T gv = fl * gravity_now<T>(&B.g, 0, xd, rtt + xd * xd);
        const bool so = solid_at(g, centre(g, 0, s), yc, zc);
        const T rho = r0 + cu[0];
        const T ir = trcp(rho);
        T q[5];
        q[0] = cu[0];
        q[1] = cu[1] * ir;
        q[2] = cu[2] * ir;
        q[3] = cu[3] * ir;
        q[4] = gm1 * (cu[4] - T(0.5) * (cu[1] * q[1] + cu[2] * q[2] + cu[3] * q[3]));
        T c, ic;
        sound(gam * (pb + q[4]) * ir, c, ic);
        T fk = T(0);
        if constexpr (FLAT) {
            // the flattening coefficient of this lane's cell (the same FP64
            // formulas as the flattening kernels): pressures three cells
            // each side and velocities two, inside the segment for every
            // cell whose parabola an owned cell's update uses (the normal
            // momentum of a wall image is flipped already)
            double p, u;
            flat_pu(fr0, fp0, (double)cu[0], (double)cu[1], (double)cu[2], (double)cu[3], (double)cu[4], g.gamma,
                    0, 1.0, p, u);
            const double pm1 = from_left(p), pp1 = from_right(p);
            const double pm2 = from_left(pm1), pp2 = from_right(pp1);
            const double um1 = from_left(u), up1 = from_right(u);
            const double r = flat_raw(pm2, pm1, pp1, pp2, um1, up1);
            fk = T(flat_pick(pm1, pp1, from_left(r), r, from_right(r)));
        }

        // (2) face values at i+1/2, second differences, limited slopes
        T qf[5], d2[5], sm[5], flm[5];
        T qp1[5];
#pragma unroll
        for (int vv = 0; vv < 5; ++vv) {
            const T qm1 = from_left(q[vv]);
            qp1[vv] = from_right(q[vv]);
            const T qp2 = from_right(qp1[vv]);
            qf[vv] = face4(qm1, q[vv], qp1[vv], qp2);
            d2[vv] = (qm1 + qp1[vv]) - T(2) * q[vv];
            sm[vv] = limited_slope(qm1, q[vv], qp1[vv]);
        }
        T r0f, p0f;
        {
            T rm = from_left(r0), rp = from_right(r0), rp2 = from_right(rp);
            T pm = from_left(pb), pp = from_right(pb), pp2 = from_right(pp);
            r0f = face4(rm, r0, rp, rp2);
            p0f = face4(pm, pb, pp, pp2);
        }
#pragma unroll
        for (int vv = 0; vv < 5; ++vv) flm[vv] = face_limited(q[vv], qp1[vv], sm[vv], from_right(sm[vv]));

        // (3) parabolas of cell i and tracing
        const bool own = lane >= NG && lane < NG + kXOut && i < nx;
        T qL[5], qR[5], dqv[5], q6[5];
#pragma unroll
        for (int vv = 0; vv < 5; ++vv) {
            T l, r;
            bool con = parabola(g.smooth_detect, q[vv], from_left(qf[vv]), qf[vv],
                                from_left(flm[vv]), flm[vv], from_left(d2[vv]), d2[vv],
                                from_right(d2[vv]), l, r);
            if (con && own && !so) ++c_uns;
            if constexpr (FLAT) {
                l = fk * q[vv] + (T(1) - fk) * l;
                r = fk * q[vv] + (T(1) - fk) * r;
            }
            qL[vv] = l; qR[vv] = r;
            dqv[vv] = r - l;
            q6[vv] = T(6) * (q[vv] - T(0.5) * (l + r));
        }
        St<T> TL, TR;
        const T r0fL = from_left(r0f), p0fL = from_left(p0f);
        trace_cell(qL, qR, dqv, q6, rho, ir, c, ic, q[1], q[0], gv, r0fL, r0f, p0fL, p0f, nu, hdt, rdx, TL, TR);

        // (4) Riemann problem and fluxes at face i+1/2
        T F[5], sg;
        {
            St<T> Rs = from_right(TR);
            bool sb = from_right_i((int)so) != 0;
            bool cnt = face_flux(TL, Rs, so, sb, r0f, p0f, gam, gfac, nu, F, sg);
            bool own_face = (own && i >= 0) || (seg == 0 && lane == NG - 1);
            if (cnt && own_face) ++c_rie;
            if constexpr (DISS) {
                // shock dissipation across a face between fluid cells; the
                // neighbour's divergence is read on every lane (a DPP read
                // from a lane masked off by a branch would not return the
                // neighbour's value), then the wall faces are zeroed
                const T dvr = from_right(dv);
                const T nv = (so || sb) ? T(0) : a.dissk * tmax(T(0), T(-0.5) * (dv + dvr));
#pragma unroll
                for (int vv = 0; vv < 5; ++vv) F[vv] = F[vv] + nv * (cu[vv] - from_right(cu[vv]));
            }
        }
        T Fl[5];
#pragma unroll
        for (int vv = 0; vv < 5; ++vv) Fl[vv] = from_left(F[vv]);
        const T sgl = from_left(sg);

        // (5) PPB: limit this cell's profile, slab at face i+1/2, update
        T L = T(1) + (sg - sgl);
        T pql[10];
#pragma unroll
        for (int v = 0; v < 10; ++v) pql[v] = pq[v];
        {
            bool hit = fv_limit(pq[0], pql[1], pql[2]);
            if (hit && own && !so) ++c_lim;
        }
        T G[10];
        {
            T dn[10];
#pragma unroll
            for (int v = 0; v < 10; ++v) dn[v] = from_right(pql[v]);
            const T Ln = from_right(L);
            // donor: this cell for a positive face velocity, else the right
            // neighbour mirrored; a zero velocity gives a zero slab
            const bool pos = sg > T(0);
#pragma unroll
            for (int v = 0; v < 10; ++v) {
                const T f = (v == 1 || v == 4 || v == 6) ? -dn[v] : dn[v];
                dn[v] = pos ? pql[v] : f;
            }
            slab(dn, sg, pos ? L : Ln, G);
        }
        T Gl[10];
#pragma unroll
        for (int v = 0; v < 10; ++v) Gl[v] = from_left(G[v]);

        {
            // stores of the owned cells; the others are switched off by
            // index; a solid cell keeps its state
            T hn[5], o[10];
            hydro_update(cu, Fl, F, nu, dt, gv, hn);
            ppb_update(pql, sg - sgl, T(0.5) * (sgl + sg), Gl, G, o);
            if (a.heat) hn[4] = hn[4] + heating_now<T>(&B.g, xt2, rtt + xd * xd) * dt;
#pragma unroll
            for (int vv = 0; vv < 5; ++vv) hn[vv] = so ? cu[vv] : hn[vv];
#pragma unroll
            for (int v = 0; v < 10; ++v) o[v] = so ? pq[v] : o[v];
            const unsigned io = own ? (unsigned)i : kNoIdx;
            T *outr = a.out + row;
            auto fo = [&](int q) { return rsrc(outr + opaque_s(nc) * q, nx); };
            bst(fo(RHO), io, hn[0]);
            bst(fo(MX), io, hn[1]);
            bst(fo(MY), io, hn[2]);
            bst(fo(MZ), io, hn[3]);
            bst(fo(EN), io, hn[4]);
#pragma unroll
            for (int v = 0; v < 10; ++v) bst(fo(AI::ppb(v)), io, o[v]);
            // the next step's CFL reduction from the values just written:
            // the exact FP64 speed only where the bound reaches the band
            // below the last maximum (in few waves), with its FP64 base
            if (a.cfl) {
                const bool need = own && !so &&
                                  speed_may_reach(r0, pb, hn[0], hn[1], hn[2], hn[3], hn[4], gam, gm1, a.cthr);
                if (__ballot(need)) {
                    const unsigned ic = need ? (unsigned)s : kNoIdx;
                    const double br0 = bld<double>(rsrc(a.r064 + row, nx), ic);
                    const double bp0 = bld<double>(rsrc(a.p064 + row, nx), ic);
                    if (need) {
                        bool bd;
                        const double sp = cell_speed(br0, bp0, (double)hn[0], (double)hn[1], (double)hn[2],
                                                     (double)hn[3], (double)hn[4], g.gamma, bd);
                        if (bd) cbad = true;
                        else cmax = fmax(cmax, sp);
                    }
                }
            }
        }
      }
      rowi = nrow;
      rx0 = nx0;
      rns = nns;
    }
    if (a.cfl) cfl_commit(b.work, m.brick, cmax, cbad);
    count_commit(a.counters, c_lim, c_uns, c_rie);
}

template <typename T, bool DISS, bool FLAT>
__global__ __launch_bounds__(256)
void sweep_x_kernel(BatchArgs<T> b)
{
    const BlockMap m = b.map[blockIdx.x];
    x_wave<T, DISS, FLAT>(b, m, m.local * (int)(blockDim.x >> 6) +
                                    __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)));
}

// The x pass uses the lanes-along-x kernel unless the shape asks for the
// marching kernel (x_rows = 0; both compute the same pass).
static bool x_lanes(const PassShape &sh) { return sh.x_rows > 0; }

int pass_blocks(const Geom &g, int axis, const PassShape &sh)
{
    if (axis == 0 && x_lanes(sh)) {
        const int nseg = (g.n[0] + kXOut - 1) / kXOut;
        const long items = (long)g.n[1] * g.n[2] * nseg;
        const long nw = (items + x_run(nseg, sh.x_rows) - 1) / x_run(nseg, sh.x_rows);   // whole rows per wave
        return (int)((nw + sh.x_waves - 1) / sh.x_waves);
    }
    const long nw = march_waves_per_chunk(g, axis);
    return (int)(march_chunks(g.n[axis], sh.march_chunk) * ((nw + sh.march_waves - 1) / sh.march_waves));
}

// Fluid cells of a pencil along `axis` whose transverse centre coordinates
// are t1, t2, estimated from the sphere's chord (for ordering work only):
// the index interval [lo, hi) it covers, clipped to the grid.
static void chord(const Geom &g, int axis, double t1, double t2, double &lo, double &hi)
{
    const int n = g.n[axis];
    lo = 0.0;
    hi = n;
    if (!g.sphere) return;
    const double rt2 = t1 * t1 + t2 * t2, R2 = g.sphere_r * g.sphere_r;
    if (!(rt2 < R2)) { lo = hi = 0.0; return; }
    const double h = std::sqrt(R2 - rt2) / g.dx, mid = -g.origin[axis] / g.dx;
    lo = std::max(0.0, mid - h - 1.0);
    hi = std::min((double)n, mid + h + 1.0);
}

static double centre_h(const Geom &g, int axis, int i) { return g.origin[axis] + ((double)i + 0.5) * g.dx; }

double pass_block_cost(const Geom &g, int axis, const PassShape &sh, int local)
{
    if (axis == 0 && x_lanes(sh)) {
        // the x rows of the block's waves: segments of 56 cells over each
        // row's fluid cells
        const int nseg = (g.n[0] + kXOut - 1) / kXOut;
        const long items = (long)g.n[1] * g.n[2] * nseg;
        const long run = x_run(nseg, sh.x_rows);
        double cost = 0.0;
        for (int w = 0; w < sh.x_waves; ++w) {
            const long it0 = ((long)local * sh.x_waves + w) * run;
            for (long it = it0; it < std::min(it0 + run, items); it += nseg) {
                const long r = it / nseg;
                double lo, hi;
                chord(g, 0, centre_h(g, 1, (int)(r % g.n[1])), centre_h(g, 2, (int)(r / g.n[1])), lo, hi);
                if (hi > lo) cost += std::ceil((hi - lo) / kXOut) * (kXOut + 2 * NG);
            }
        }
        return cost;
    }
    // marching waves: the widest pencil's fluid cells inside the chunk, plus
    // the 8 cells read beyond it (sampled on a few of the wave's pencils)
    const int ca = (axis == 0) ? 1 : 0;
    const int cb = 3 - axis - ca;
    const int na = g.n[ca];
    const int nchk = march_chunks(g.n[axis], sh.march_chunk);
    const int clen = sh.march_chunk > 0 ? sh.march_chunk : g.n[axis];
    const int ck = local % nchk, rest = local / nchk;
    const int nblk_a = (na + 63) / 64;
    const double clo = ck * clen, chi = std::min(clo + clen, (double)g.n[axis]);
    double cost = 0.0;
    for (int w = 0; w < sh.march_waves; ++w) {
        const long wq = (long)rest * sh.march_waves + w;
        double best = -1.0;
        for (int l = 0; l < 64; l += 9) {
            long la, lb;
            if (march_packed(g, axis)) {
                const long rows = march_rows(g, axis);
                if (l >= rows * na) break;
                la = l % na;
                lb = wq * rows + l / na;
                if (lb >= g.n[cb]) break;
            } else {
                la = (wq % nblk_a) * 64 + l;
                lb = wq / nblk_a;
                if (lb >= g.n[cb] || la >= na) break;
            }
            double t[3];
            t[ca] = centre_h(g, ca, (int)la);
            t[cb] = centre_h(g, cb, (int)lb);
            double lo, hi;
            chord(g, axis, t[(axis + 1) % 3], t[(axis + 2) % 3], lo, hi);
            best = std::max(best, std::min(hi, chi) - std::max(lo, clo));
        }
        if (best > 0.0) cost += best + 2 * NG;
    }
    return cost;
}

// ---------------------------------------------------------------------
// Persistent step: one launch of resident waves for the three passes of
// every brick and the dt of the step (stages and waits as declared with
// launch_step).  An item is one wave's share of a stage: the same code and
// the same block maps as the per-stage launches, so the result is the same
// bit for bit.
// ---------------------------------------------------------------------

template <typename T>
struct StepArgs {
    BatchArgs<T> common;          // what the three passes share (arenas, maps and flags set per pass)
    T *a0;                        // the state the step starts from; passes go a0 -> a1 -> a0 -> a1
    T *a1;
    const BlockMap *map0, *map1, *map2;
    const BlockMap *cmap;         // CFL blocks (redo reduction)
    const int *need;              // [stage * nb + brick]
    unsigned long long *cnt;      // [nb] items done per brick; then next item, abort flag
    double *dt;
    double cfl;
    long first[kStepStages + 1];  // item where each stage starts
    int ax0, ax1, ax2;            // pass axes in step order
    int w0, w1, w2;               // waves per block of each pass's map
    int nb;
    int heat;
    int skip_first;               // first pass: solid cells alike in both arenas
    int ready;                    // the maxima in work[] describe a0: stages 0-2 give dt
};

// Bounded wait: a wait gives up after 0.25 s of real time (the 100 MHz
// real-time counter); a wait in a working step lasts at most one pass.
constexpr unsigned long long kStepWaitTicks = 25000000ull;

__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Wait (the whole wave, polling one word) until *c reaches `need` or the
// step is abandoned, then acquire: the writes of the counted items are
// visible to this wave.
__device__ __forceinline__ void step_wait(unsigned long long *c, unsigned long long need, unsigned long long *abort)
{
    if (need == 0) return;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        if (uniform_u64(__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >= need) break;
        if (uniform_u64(__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) break;
        if (__builtin_amdgcn_s_memrealtime() - t0 > kStepWaitTicks) {
            if ((threadIdx.x & 63) == 0) __hip_atomic_store(abort, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(4);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Release this wave's writes, then count its item done.
__device__ __forceinline__ void step_done(unsigned long long *c)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_add(c, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__global__ __launch_bounds__(64, sizeof(T) == 4 ? 2 : 1)
void step_kernel(StepArgs<T> P)
{
    unsigned long long *ctl = P.cnt + P.nb;
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned long long it = 0;
        if (lane == 0) it = __hip_atomic_fetch_add(&ctl[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        it = uniform_u64(it);
        if (it >= (unsigned long long)P.first[kStepStages]) break;
        // the stage: the last one starting at or before the item (an empty
        // stage starts where the next one does)
        int s = 0;
        long s0 = 0;
#pragma unroll
        for (int k = 1; k < kStepStages; ++k)
            if (it >= (unsigned long long)P.first[k]) {
                s = k;
                s0 = P.first[k];
            }
        const long j = (long)it - s0;
        const int p = s - 4;                             // pass in step order (stages 4-6)
        const int w = p == 0 ? P.w0 : (p == 1 ? P.w1 : P.w2);
        const BlockMap *pm = p == 0 ? P.map0 : (p == 1 ? P.map1 : P.map2);
        BlockMap m{ (int)j, 0 };
        if (s == 1) m = P.cmap[j >> 2];
        else if (s >= 4) m = pm[j / w];
        const int brick = __builtin_amdgcn_readfirstlane(m.brick);
        m.brick = brick;
        m.local = __builtin_amdgcn_readfirstlane(m.local);
        step_wait(&P.cnt[brick], (unsigned long long)P.need[(long)s * P.nb + brick], &ctl[1]);
        const BatchArgs<T> &c0 = P.common;
        if (s == 0) {
            if (P.ready && lane == 0) cfl_check_brick(c0.bricks, brick, c0.work, const_cast<unsigned long long *>(c0.cband), P.cfl, P.dt);
        } else if (s == 1) {
            if (P.ready && c0.cband[2 * brick + 1] != 0ull)
                cfl_block_part<T>(c0.bricks, m, P.a0, c0.base64, c0.work, (int)(j & 3) * 64 + lane, 256);
        } else if (s == 2) {
            if (P.ready && lane == 0) cfl_redo_finish_brick(c0.bricks, brick, c0.work, const_cast<unsigned long long *>(c0.cband), P.cfl, P.dt);
        } else if (s == 3) {
            if (lane == 0) cfl_arm_brick(c0.work, const_cast<unsigned long long *>(c0.cband), brick);
        } else {
            BatchArgs<T> b = c0;
            b.in = p == 1 ? P.a1 : P.a0;
            b.out = p == 1 ? P.a0 : P.a1;
            b.map = pm;
            b.cfl = p == 2 ? 1 : 0;
            b.heat = p == 2 ? P.heat : 0;
            b.skip = p == 0 ? P.skip_first : c0.skip;
            const int ax = p == 0 ? P.ax0 : (p == 1 ? P.ax1 : P.ax2);
            const int wv = (int)(j % w);
            if (ax == 0) x_wave<T, false, false>(b, m, m.local * w + wv);
            else if (ax == 1) march_wave<T, 1, false, false>(b, m, wv, w);
            else march_wave<T, 2, false, false>(b, m, wv, w);
        }
        step_done(&P.cnt[brick]);
    }
}

bool step_eligible(const PassShape &sh) { return sh.x_rows > 0; }

long step_stage_units(const PassShape &sh, int stage, const int order[3], const int nblk_b[3], int ncb_b)
{
    switch (stage) {
    case 0: case 2: case 3: return 1;
    case 1: return 4L * ncb_b;
    default: {
        const int ax = order[stage - 4];
        return (long)nblk_b[stage - 4] * (ax == 0 ? sh.x_waves : sh.march_waves);
    }
    }
}

template <typename T>
int step_workers()
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, step_kernel<T>, 64, 0) != hipSuccess) return 0;
    return cus * per;
}

template <typename T>
hipError_t launch_step(const PassShape &sh, const Brick *bricks, int nb, const int order[3],
                       const BlockMap *const maps[3], const int nblocks[3], const BlockMap *cmap, int ncblocks,
                       const int *need, unsigned long long *cnt, T *a0, T *a1, const T *base,
                       double *dt, unsigned long long *counters, int heat, const double *base64,
                       unsigned long long *work, unsigned long long *cband, int skip_first, int skip, int ready,
                       double cfl, int workers, hipStream_t st)
{
    if (nb <= 0 || workers <= 0 || !step_eligible(sh)) return hipErrorInvalidValue;
    StepArgs<T> P{};
    P.common = BatchArgs<T>{ bricks, nullptr, nullptr, nullptr, base, dt, counters, base64, work, cband,
                             nullptr, 0.0, nullptr, 0, 0, skip, sh.march_chunk, sh.x_rows };
    P.a0 = a0;
    P.a1 = a1;
    P.map0 = maps[0];
    P.map1 = maps[1];
    P.map2 = maps[2];
    P.cmap = cmap;
    P.need = need;
    P.cnt = cnt;
    P.dt = dt;
    P.cfl = cfl;
    P.ax0 = order[0];
    P.ax1 = order[1];
    P.ax2 = order[2];
    P.w0 = order[0] == 0 ? sh.x_waves : sh.march_waves;
    P.w1 = order[1] == 0 ? sh.x_waves : sh.march_waves;
    P.w2 = order[2] == 0 ? sh.x_waves : sh.march_waves;
    P.nb = nb;
    P.heat = heat;
    P.skip_first = skip_first;
    P.ready = ready;
    const long units[kStepStages] = { nb, 4L * ncblocks, nb, nb, (long)nblocks[0] * P.w0,
                                      (long)nblocks[1] * P.w1, (long)nblocks[2] * P.w2 };
    P.first[0] = 0;
    for (int s = 0; s < kStepStages; ++s) P.first[s + 1] = P.first[s] + units[s];
    const long grid = std::min<long>(workers, P.first[kStepStages]);
    hipLaunchKernelGGL((step_kernel<T>), dim3((unsigned)grid), dim3(64), 0, st, P);
    return hipGetLastError();
}

template hipError_t launch_step<float>(const PassShape &, const Brick *, int, const int[3], const BlockMap *const[3],
                                       const int[3], const BlockMap *, int, const int *, unsigned long long *,
                                       float *, float *, const float *, double *, unsigned long long *, int,
                                       const double *, unsigned long long *, unsigned long long *, int, int, int,
                                       double, int, hipStream_t);
template hipError_t launch_step<double>(const PassShape &, const Brick *, int, const int[3],
                                        const BlockMap *const[3], const int[3], const BlockMap *, int, const int *,
                                        unsigned long long *, double *, double *, const double *, double *,
                                        unsigned long long *, int, const double *, unsigned long long *,
                                        unsigned long long *, int, int, int, double, int, hipStream_t);
template int step_workers<float>();
template int step_workers<double>();

template <typename T, bool D, bool F>
static void launch_pass_kernel(int axis, bool xl, int nblocks, const PassShape &sh, hipStream_t st,
                               const BatchArgs<T> &a)
{
    if (xl) {
        hipLaunchKernelGGL((sweep_x_kernel<T, D, F>), dim3(nblocks), dim3(64 * sh.x_waves), 0, st, a);
        return;
    }
    dim3 grid(nblocks), block(64 * sh.march_waves);
    switch (axis) {
    case 0: hipLaunchKernelGGL((sweep_kernel<T, 0, D, F>), grid, block, 0, st, a); break;
    case 1: hipLaunchKernelGGL((sweep_kernel<T, 1, D, F>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((sweep_kernel<T, 2, D, F>), grid, block, 0, st, a); break;
    }
}

template <typename T>
hipError_t launch_sweep(int axis, const PassShape &sh, const Brick *bricks, const BlockMap *map,
                        int nblocks, const T *in, T *out, const T *base, const double *dt,
                        unsigned long long *counters, int heat, const double *base64,
                        unsigned long long *work, const unsigned long long *cband, const T *div, double dissk,
                        const T *flat, int cfl, int skip, hipStream_t st)
{
    if (nblocks <= 0) return hipErrorInvalidValue;
    const bool diss = dissk > 0.0 && div;
    BatchArgs<T> a{bricks, map, in, out, base, dt, counters, base64, work, cband, diss ? div : nullptr,
                   dissk, flat, heat, cfl, skip, sh.march_chunk, sh.x_rows};
    const bool xl = axis == 0 && x_lanes(sh);
    if (diss && flat) launch_pass_kernel<T, true, true>(axis, xl, nblocks, sh, st, a);
    else if (diss) launch_pass_kernel<T, true, false>(axis, xl, nblocks, sh, st, a);
    else if (flat) launch_pass_kernel<T, false, true>(axis, xl, nblocks, sh, st, a);
    else launch_pass_kernel<T, false, false>(axis, xl, nblocks, sh, st, a);
    return hipGetLastError();
}

template hipError_t launch_sweep<float>(int, const PassShape &, const Brick *, const BlockMap *, int,
                                        const float *, float *, const float *, const double *,
                                        unsigned long long *, int, const double *, unsigned long long *,
                                        const unsigned long long *, const float *, double, const float *, int,
                                        int, hipStream_t);
template hipError_t launch_sweep<double>(int, const PassShape &, const Brick *, const BlockMap *, int,
                                         const double *, double *, const double *, const double *,
                                         unsigned long long *, int, const double *, unsigned long long *,
                                         const unsigned long long *, const double *, double, const double *, int,
                                         int, hipStream_t);

}  // namespace ppmb
