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

#include <cstdlib>

namespace ppmb {

// Per-brick view handed to the pencil code: the brick's state, output and
// base fields, its dt and cell count.
template <typename T>
struct SweepArgs {
    const T *in;          // 15 fields, stride ncell
    T *out;
    const T *rho0;        // base state, working precision
    const T *p0;
    const double *dtp;    // this brick's dt
    unsigned long long *counters;   // limiter, unsmooth, riemann
    long ncell;
    int heat;             // 1: add the heating source after the update
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
    int heat;
};

template <typename T>
__device__ __forceinline__ SweepArgs<T> brick_args(const BatchArgs<T> &b, const Brick &B)
{
    return SweepArgs<T>{b.in + B.off, b.out + B.off, b.base + B.boff, b.base + B.boff + B.ncell,
                        b.dt + B.dti, b.counters, B.ncell, b.heat};
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

// March one pencil; la / lb index it across the lane and block axes.
template <typename T, int AX>
__device__ void march(const Geom &g, const SweepArgs<T> &a, int la, int lb,
                      unsigned long long &c_lim, unsigned long long &c_uns, unsigned long long &c_rie)
{
    using AI = AxisInfo<AX>;
    const int nx = g.n[0], ny = g.n[1];
    const int n = g.n[AX];
    const int ca = (AX == 0) ? 1 : 0;
    const int cb = 3 - AX - ca;
    int ijk0[3];
    ijk0[ca] = la; ijk0[cb] = lb; ijk0[AX] = 0;
    const long stride[3] = { 1, (long)nx, (long)nx * ny };
    const long base = ijk0[0] * stride[0] + ijk0[1] * stride[1] + ijk0[2] * stride[2];
    const long sAX = stride[AX];
    const double xt[3] = { centre(g, 0, ijk0[0]), centre(g, 1, ijk0[1]), centre(g, 2, ijk0[2]) };
    // transverse part of |x|^2 and the fluid interval of this pencil
    const T xt1 = T(xt[AI::t1]), xt2 = T(xt[AI::t2]);
    const T rtt = xt1 * xt1 + xt2 * xt2;
    int flo, fhi;
    fluid_interval(g, AX, xt, flo, fhi);
    const T ox = T(g.origin[AX]), dxT = T(g.dx);

    const double dt64 = *a.dtp;
    const T dt = T(dt64), nu = T(dt64 / g.dx), hdt = T(0.5 * dt64), rdx = T(1.0 / g.dx);
    const T gam = T(g.gamma), gm1 = T(g.gamma - 1.0), gfac = T(g.gamma / (g.gamma - 1.0));
    const int bc = g.bc[AX];
    const T *in = a.in;
    const long nc = a.ncell;

    // --- register window ---------------------------------------------
    T q[5][5];            // primitives rho', u, v, w, p' of cells k-4..k
    T rr[3], cr[3];       // rho, c of cells k-2..k
    T b0[4], b1[4];       // base rho0, p0 of cells k-3..k
    T gr[4];              // gravity along the pass, cells k-3..k
    T cu[4][5];           // conserved rho', mn, mt1, mt2, E' of cells k-3..k
    bool sol[5];          // solid flags of cells k-4..k
    T qf[2][5], r0f[2], p0f[2];   // faces (k-3)+1/2 and (k-2)+1/2
    T sm[3][5];           // limited slopes of cells k-3..k-1
    T d2[3][5];           // second differences of cells k-3..k-1
    T flm[2][5];          // limited-slope face values at (k-3)+1/2, (k-2)+1/2
    St<T> TLp;            // right-face state of cell k-3
    T Fp[5];              // fluxes at face (k-4)+1/2
    T sg1 = T(0), sg2 = T(0);     // sigma at faces (k-4)+1/2, (k-5)+1/2
    T hyd[5];             // updated hydro of cell k-4
    T pq[10], pqp[10];    // fv coefficients of cells k-3 (this step) and k-4 (limited)
    T Lp = T(1);          // Lagrangian length of cell k-4
    T Gp[10];             // slab at face (k-5)+1/2
    for (int v = 0; v < 5; ++v) { Fp[v] = T(0); hyd[v] = T(0); }
    for (int v = 0; v < 10; ++v) { pq[v] = T(0); pqp[v] = T(0); Gp[v] = T(0); }
    TLp = St<T>{T(0), T(0), T(0), T(0), T(0)};
    for (int c = 0; c < 4; ++c) { gr[c] = T(0); b0[c] = T(0); b1[c] = T(0); }
    for (int c = 0; c < 5; ++c) sol[c] = false;

    for (int k = -NG; k < n + NG; ++k) {
        // ---- (1) load cell k and form its primitives (base added back, Sec. 1)
        {
            int fl = 1;
            int s = k;
            if (k < 0 || k >= n) s = bc_source(k, n, bc, fl);
            long ci = base + s * sAX;
            T rp = in[RHO * nc + ci];
            T mn = T(fl) * in[(MX + AX) * nc + ci];
            T m1 = in[(MX + AI::t1) * nc + ci];
            T m2 = in[(MX + AI::t2) * nc + ci];
            T ep = in[EN * nc + ci];
            T r0 = a.rho0[ci], pb = a.p0[ci];
            T xd = ox + (T(s) + T(0.5)) * dxT;
            T gv = T(fl) * gravity<T>(g, AX, xd, rtt + xd * xd);
            bool so = s < flo || s > fhi;
            T rho = r0 + rp;
            T ir = trcp(rho);
            T u = mn * ir, v = m1 * ir, w = m2 * ir;
            T pp = gm1 * (ep - T(0.5) * (mn * u + m1 * v + m2 * w));
            T c = tsqrt(gam * (pb + pp) * ir);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int vv = 0; vv < 5; ++vv) q[r][vv] = q[r + 1][vv];
            q[4][0] = rp; q[4][1] = u; q[4][2] = v; q[4][3] = w; q[4][4] = pp;
            rr[0] = rr[1]; rr[1] = rr[2]; rr[2] = rho;
            cr[0] = cr[1]; cr[1] = cr[2]; cr[2] = c;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                b0[r] = b0[r + 1]; b1[r] = b1[r + 1]; gr[r] = gr[r + 1];
#pragma unroll
                for (int vv = 0; vv < 5; ++vv) cu[r][vv] = cu[r + 1][vv];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) sol[r] = sol[r + 1];
            b0[3] = r0; b1[3] = pb; gr[3] = gv; sol[4] = so;
            cu[3][0] = rp; cu[3][1] = mn; cu[3][2] = m1; cu[3][3] = m2; cu[3][4] = ep;
        }
        // fv coefficients of cell k-3 (donors -1..n)
        if (k - 3 >= -1) {
            int fl = 1;
            int s = k - 3;
            if (s < 0 || s >= n) s = bc_source(k - 3, n, bc, fl);
            long ci = base + s * sAX;
#pragma unroll
            for (int v = 0; v < 10; ++v) {
                T val = in[AI::ppb(v) * nc + ci];
                pq[v] = AI::odd(v) ? T(fl) * val : val;
            }
        }
        // ---- (2) interface values at face (k-2)+1/2 (cells k-3..k)
        if (k >= -1) {
#pragma unroll
            for (int vv = 0; vv < 5; ++vv) { qf[0][vv] = qf[1][vv]; qf[1][vv] = face4(q[1][vv], q[2][vv], q[3][vv], q[4][vv]); }
            r0f[0] = r0f[1]; r0f[1] = face4(b0[0], b0[1], b0[2], b0[3]);
            p0f[0] = p0f[1]; p0f[1] = face4(b1[0], b1[1], b1[2], b1[3]);
        }
        // ---- (3) limited slope and second difference of cell k-1; the
        //          limited-slope face value at (k-2)+1/2
        if (k >= -2) {
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
        if (k < 0) continue;
        // ---- (4) parabolas of cell k-2, constrained only where the 5-cell
        //          window is not smooth (Sec. 1), blended over the graded
        //          band; tracing (CW84 Sec. 3)
        St<T> TL, TR;
        {
            const bool interior = (k - 2 >= 0) && (k - 2 < n);
            T qL[5], qR[5], dq[5], q6[5];
#pragma unroll
            for (int vv = 0; vv < 5; ++vv) {
                T l, r;
                bool con = parabola(g.smooth_detect, q[2][vv], qf[0][vv], qf[1][vv], flm[0][vv], flm[1][vv],
                                    d2[0][vv], d2[1][vv], d2[2][vv], l, r);
                if (con && interior) ++c_uns;
                qL[vv] = l; qR[vv] = r;
                dq[vv] = r - l;
                q6[vv] = T(6) * (q[2][vv] - T(0.5) * (l + r));
            }
            trace_cell(qL, qR, dq, q6, rr[0], cr[0], q[2][1], q[2][0], gr[1], r0f[0], r0f[1], p0f[0],
                       p0f[1], nu, hdt, rdx, TL, TR);
        }
        // ---- (5) Riemann problem and fluxes at face (k-3)+1/2
        T F[5] = { T(0), T(0), T(0), T(0), T(0) };
        T sg = T(0);
        if (k >= 1) {
            bool cnt = face_flux(TLp, TR, sol[1], sol[2], r0f[0], p0f[0], gam, gfac, nu, F, sg);
            if (cnt && k - 3 >= -1 && k - 3 < n) ++c_rie;
        }
        TLp = TL;
        // ---- (6) conservative update of cell k-3 (written one step later)
        T hn[5] = { T(0), T(0), T(0), T(0), T(0) };
        const int cu_ = k - 3;
        if (cu_ >= 0 && cu_ < n) {
            if (sol[1]) {
                for (int vv = 0; vv < 5; ++vv) hn[vv] = cu[0][vv];
            } else {
                hydro_update(cu[0], Fp, F, nu, dt, gr[0], hn);
            }
        }
        // ---- (7) PPB: donor k-3, slab at face (k-4)+1/2, update cell k-4
        if (k >= 2) {
            T Ld = T(1) + (sg - sg1);
            T l1 = pq[1], l2 = pq[2];
            bool hit = fv_limit(pq[0], l1, l2);
            if (hit && k - 3 >= 0 && k - 3 < n && !sol[1]) ++c_lim;
            T pql[10];
#pragma unroll
            for (int v = 0; v < 10; ++v) pql[v] = pq[v];
            pql[1] = l1; pql[2] = l2;
            T G[10];
            if (k >= 3) {
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
                if (cw >= 0 && cw < n) {
                    long ci = base + cw * sAX;
                    T o[10];
                    const bool solid_w = sol[0];
                    if (solid_w) {
#pragma unroll
                        for (int v = 0; v < 10; ++v) o[v] = in[AI::ppb(v) * nc + ci];
                    } else {
                        ppb_update(pqp, sg1 - sg2, T(0.5) * (sg2 + sg1), Gp, G, o);
                    }
                    T e = hyd[4];
                    if (a.heat && !solid_w) {
                        T xd = ox + (T(cw) + T(0.5)) * dxT;
                        T zc = AX == 2 ? xd : T(xt[2]);
                        e = e + heating<T>(g, zc, rtt + xd * xd) * dt;
                    }
                    a.out[RHO * nc + ci] = hyd[0];
                    a.out[(MX + AX) * nc + ci] = hyd[1];
                    a.out[(MX + AI::t1) * nc + ci] = hyd[2];
                    a.out[(MX + AI::t2) * nc + ci] = hyd[3];
                    a.out[EN * nc + ci] = e;
#pragma unroll
                    for (int v = 0; v < 10; ++v) a.out[AI::ppb(v) * nc + ci] = o[v];
                }
#pragma unroll
                for (int v = 0; v < 10; ++v) Gp[v] = G[v];
            }
#pragma unroll
            for (int v = 0; v < 10; ++v) pqp[v] = pql[v];
            Lp = Ld;
        }
        sg2 = sg1; sg1 = sg;
#pragma unroll
        for (int vv = 0; vv < 5; ++vv) { Fp[vv] = F[vv]; hyd[vv] = hn[vv]; }
    }
}

// Marching kernel: each wave covers 64 pencils (lanes across x for the y
// and z passes, across y for the x pass); a block holds blockDim/64 waves
// on consecutive rows of the other transverse axis.
// FP32: at most 256 VGPRs, two waves per SIMD; FP64 needs the full file.
template <typename T, int AX>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1)
void sweep_kernel(BatchArgs<T> b)
{
    const BlockMap m = b.map[blockIdx.x];
    const Brick &B = b.bricks[m.brick];
    const Geom g = B.g;
    const SweepArgs<T> a = brick_args(b, B);
    const int ca = (AX == 0) ? 1 : 0;
    const int cb = 3 - AX - ca;
    const int waves = blockDim.x >> 6;
    const int nblk_a = (g.n[ca] + 63) / 64;
    const int la = (m.local % nblk_a) * 64 + (threadIdx.x & 63);
    const int lb = (m.local / nblk_a) * waves + (threadIdx.x >> 6);
    unsigned long long c_lim = 0, c_uns = 0, c_rie = 0;
    if (la < g.n[ca] && lb < g.n[cb]) march<T, AX>(g, a, la, lb, c_lim, c_uns, c_rie);
    // event counters: one atomic per wave and counter
    unsigned long long s0 = c_lim, s1 = c_uns, s2 = c_rie;
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_down(s0, off);
        s1 += __shfl_down(s1, off);
        s2 += __shfl_down(s2, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (s0) atomicAdd(&a.counters[0], s0);
        if (s1) atomicAdd(&a.counters[1], s1);
        if (s2) atomicAdd(&a.counters[2], s2);
    }
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

// Neighbour values inside the wave by DPP whole-wave shifts (wave_shr:1,
// wave_shl:1): a VALU move, no LDS round trip.  The lane at the wave's edge
// keeps its own value, so every lane holds a physical state.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
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
    int s, fl;
};

template <typename T>
__device__ __forceinline__ void x_load(const T *in, const T *rho0, const T *p0, long nc, long row,
                                       int nx, int bc, int i, XIn<T> &o)
{
    using AI = AxisInfo<0>;
    int fl = 1;
    int s = i;
    if (i < 0 || i >= nx) s = bc_source(i, nx, bc, fl);
    const long ci = row + s;
    o.s = s;
    o.fl = fl;
    o.cu[0] = in[RHO * nc + ci];
    o.cu[1] = in[MX * nc + ci];
    o.cu[2] = in[MY * nc + ci];
    o.cu[3] = in[MZ * nc + ci];
    o.cu[4] = in[EN * nc + ci];
#pragma unroll
    for (int v = 0; v < 10; ++v) o.pq[v] = in[AI::ppb(v) * nc + ci];
    o.r0 = rho0[ci];
    o.pb = p0[ci];
}

// One wave owns one x-row and walks it in segments of 56 outputs; the
// loads of the next segment are issued before the current one is computed,
// so their latency hides behind the arithmetic.
template <typename T>
__global__ __launch_bounds__(256)
void sweep_x_kernel(BatchArgs<T> b)
{
    using AI = AxisInfo<0>;
    const BlockMap m = b.map[blockIdx.x];
    const Brick &B = b.bricks[m.brick];
    const Geom g = B.g;
    const SweepArgs<T> a = brick_args(b, B);
    const int lane = threadIdx.x & 63;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int rowi = m.local * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    if (rowi >= ny * nz) return;                       // whole waves only
    const int y = rowi % ny, z = rowi / ny;
    const int nseg = (nx + kXOut - 1) / kXOut;
    const long nc = a.ncell;
    const long row = (long)rowi * nx;
    const double yc = centre(g, 1, y), zc = centre(g, 2, z);
    const T xt1 = T(yc), xt2 = T(zc);
    const T rtt = xt1 * xt1 + xt2 * xt2;
    const double dt64 = *a.dtp;
    const T dt = T(dt64), nu = T(dt64 / g.dx), hdt = T(0.5 * dt64), rdx = T(1.0 / g.dx);
    const T gam = T(g.gamma), gm1 = T(g.gamma - 1.0), gfac = T(g.gamma / (g.gamma - 1.0));
    const T ox = T(g.origin[0]), dxT = T(g.dx);
    const int bc = g.bc[0];
    unsigned long long c_lim = 0, c_uns = 0, c_rie = 0;

    XIn<T> cur, nxt;
    x_load(a.in, a.rho0, a.p0, nc, row, nx, bc, -NG + lane, cur);
    for (int seg = 0; seg < nseg; ++seg) {
        const int i = seg * kXOut - NG + lane;         // this lane's cell along x
        if (seg + 1 < nseg) x_load(a.in, a.rho0, a.p0, nc, row, nx, bc, i + kXOut, nxt);

        // (1) this lane's cell: primitives, gravity, solid flag
        const int s = cur.s;
        const T fl = T(cur.fl);
        T cu[5], pq[10];
        cu[0] = cur.cu[0];
        cu[1] = fl * cur.cu[1];
        cu[2] = cur.cu[2];
        cu[3] = cur.cu[3];
        cu[4] = cur.cu[4];
#pragma unroll
        for (int v = 0; v < 10; ++v) pq[v] = AI::odd(v) ? fl * cur.pq[v] : cur.pq[v];
        const T r0 = cur.r0, pb = cur.pb;
        const T xd = ox + (T(s) + T(0.5)) * dxT;
        const T gv = fl * gravity<T>(g, 0, xd, rtt + xd * xd);
        const bool so = solid_at(g, centre(g, 0, s), yc, zc);
        const T rho = r0 + cu[0];
        const T ir = trcp(rho);
        T q[5];
        q[0] = cu[0];
        q[1] = cu[1] * ir;
        q[2] = cu[2] * ir;
        q[3] = cu[3] * ir;
        q[4] = gm1 * (cu[4] - T(0.5) * (cu[1] * q[1] + cu[2] * q[2] + cu[3] * q[3]));
        const T c = tsqrt(gam * (pb + q[4]) * ir);

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
            if (con && own) ++c_uns;
            qL[vv] = l; qR[vv] = r;
            dqv[vv] = r - l;
            q6[vv] = T(6) * (q[vv] - T(0.5) * (l + r));
        }
        St<T> TL, TR;
        const T r0fL = from_left(r0f), p0fL = from_left(p0f);
        trace_cell(qL, qR, dqv, q6, rho, c, q[1], q[0], gv, r0fL, r0f, p0fL, p0f, nu, hdt, rdx, TL, TR);

        // (4) Riemann problem and fluxes at face i+1/2
        T F[5], sg;
        {
            St<T> Rs = from_right(TR);
            bool sb = from_right_i((int)so) != 0;
            bool cnt = face_flux(TL, Rs, so, sb, r0f, p0f, gam, gfac, nu, F, sg);
            bool own_face = (own && i >= 0) || (seg == 0 && lane == NG - 1);
            if (cnt && own_face) ++c_rie;
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

        if (own) {
            T hn[5], o[10];
            if (so) {
#pragma unroll
                for (int vv = 0; vv < 5; ++vv) hn[vv] = cu[vv];
#pragma unroll
                for (int v = 0; v < 10; ++v) o[v] = pq[v];
            } else {
                hydro_update(cu, Fl, F, nu, dt, gv, hn);
                ppb_update(pql, sg - sgl, T(0.5) * (sgl + sg), Gl, G, o);
                if (a.heat) hn[4] = hn[4] + heating<T>(g, xt2, rtt + xd * xd) * dt;
            }
            const long co = row + i;
            a.out[RHO * nc + co] = hn[0];
            a.out[MX * nc + co] = hn[1];
            a.out[MY * nc + co] = hn[2];
            a.out[MZ * nc + co] = hn[3];
            a.out[EN * nc + co] = hn[4];
#pragma unroll
            for (int v = 0; v < 10; ++v) a.out[AI::ppb(v) * nc + co] = o[v];
        }
        if (seg + 1 < nseg) cur = nxt;
    }
    unsigned long long s0 = c_lim, s1 = c_uns, s2 = c_rie;
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_down(s0, off);
        s1 += __shfl_down(s1, off);
        s2 += __shfl_down(s2, off);
    }
    if (lane == 0) {
        if (s0) atomicAdd(&a.counters[0], s0);
        if (s1) atomicAdd(&a.counters[1], s1);
        if (s2) atomicAdd(&a.counters[2], s2);
    }
}

// The x pass uses the lanes-along-x kernel unless PPMB_X_MARCH=1 selects
// the marching kernel (kept for comparison; both compute the same pass).
static bool x_lanes_enabled()
{
    const char *e = getenv("PPMB_X_MARCH");
    return !(e && e[0] == '1');
}

int pass_blocks(const Geom &g, int axis, const PassShape &sh)
{
    if (axis == 0 && x_lanes_enabled()) {
        const long nw = (long)g.n[1] * g.n[2];            // one wave per x-row
        return (int)((nw + sh.x_waves - 1) / sh.x_waves);
    }
    const int ca = (axis == 0) ? 1 : 0;
    const int cb = 3 - axis - ca;
    return ((g.n[ca] + 63) / 64) * ((g.n[cb] + sh.march_waves - 1) / sh.march_waves);
}

template <typename T>
hipError_t launch_sweep(int axis, const PassShape &sh, const Brick *bricks, const BlockMap *map,
                        int nblocks, const T *in, T *out, const T *base, const double *dt,
                        unsigned long long *counters, int heat, hipStream_t st)
{
    if (nblocks <= 0) return hipErrorInvalidValue;
    BatchArgs<T> a{bricks, map, in, out, base, dt, counters, heat};
    if (axis == 0 && x_lanes_enabled()) {
        hipLaunchKernelGGL((sweep_x_kernel<T>), dim3(nblocks), dim3(64 * sh.x_waves), 0, st, a);
        return hipGetLastError();
    }
    dim3 grid(nblocks), block(64 * sh.march_waves);
    switch (axis) {
    case 0: hipLaunchKernelGGL((sweep_kernel<T, 0>), grid, block, 0, st, a); break;
    case 1: hipLaunchKernelGGL((sweep_kernel<T, 1>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((sweep_kernel<T, 2>), grid, block, 0, st, a); break;
    }
    return hipGetLastError();
}

template hipError_t launch_sweep<float>(int, const PassShape &, const Brick *, const BlockMap *, int,
                                        const float *, float *, const float *, const double *,
                                        unsigned long long *, int, hipStream_t);
template hipError_t launch_sweep<double>(int, const PassShape &, const Brick *, const BlockMap *, int,
                                         const double *, double *, const double *, const double *,
                                         unsigned long long *, int, hipStream_t);

}  // namespace ppmb
