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

namespace ppmb {

template <typename T>
struct SweepArgs {
    const T *in;          // 15 fields, stride ncell
    T *out;
    const T *rho0;        // base state, working precision
    const T *p0;
    const double *dtp;    // device dt
    unsigned long long *counters;   // limiter, unsmooth, riemann, (steps)
    long ncell;
    int heat;             // 1: add the heating source after the update
};

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
            int fl;
            int s = bc_source(k, n, bc, fl);
            long ci = base + s * sAX;
            T rp = in[RHO * nc + ci];
            T mn = T(fl) * in[(MX + AX) * nc + ci];
            T m1 = in[(MX + AI::t1) * nc + ci];
            T m2 = in[(MX + AI::t2) * nc + ci];
            T ep = in[EN * nc + ci];
            T r0 = a.rho0[ci], pb = a.p0[ci];
            double xs[3] = { xt[0], xt[1], xt[2] };
            xs[AX] = centre(g, AX, s);
            T gv = T(fl) * gravity<T>(g, AX, xs[0], xs[1], xs[2]);
            bool so = solid_at(g, xs[0], xs[1], xs[2]);
            T rho = r0 + rp;
            T u = mn / rho, v = m1 / rho, w = m2 / rho;
            T pp = gm1 * (ep - T(0.5) * (mn * u + m1 * v + m2 * w));
            T c = sqrt(gam * (pb + pp) / rho);
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
            int fl;
            int s = bc_source(k - 3, n, bc, fl);
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
        // ---- (3) limited slope of cell k-1
        if (k >= -2) {
#pragma unroll
            for (int vv = 0; vv < 5; ++vv) { sm[0][vv] = sm[1][vv]; sm[1][vv] = sm[2][vv]; sm[2][vv] = limited_slope(q[2][vv], q[3][vv], q[4][vv]); }
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
                T ws = g.smooth_detect == 1 ? smooth_weight(q[0][vv], q[1][vv], q[2][vv], q[3][vv], q[4][vv])
                                            : T(g.smooth_detect == 2 ? 1 : 0);
                T l = qf[0][vv], r = qf[1][vv];
                if (ws < T(1)) {
                    T lc = face_limited(q[1][vv], q[2][vv], sm[0][vv], sm[1][vv]);
                    T rc = face_limited(q[2][vv], q[3][vv], sm[1][vv], sm[2][vv]);
                    constrain(q[2][vv], lc, rc);
                    if (ws > T(0)) { lc = lc + ws * (l - lc); rc = rc + ws * (r - rc); }
                    l = lc; r = rc;
                    if (interior) ++c_uns;
                }
                qL[vv] = l; qR[vv] = r;
                dq[vv] = r - l;
                q6[vv] = T(6) * (q[2][vv] - T(0.5) * (l + r));
            }
            const T rj = rr[0], cj = cr[0], uj = q[2][1], c2 = cj * cj;
            const T lm = uj - cj, l0 = uj, lp = uj + cj;
            const T rc2 = rj / (T(2) * cj), cr_ = cj / rj, i2c2 = T(1) / (T(2) * c2), ic2 = T(1) / c2;
            {   // right face: waves moving right
                T y = tmax(lp, T(0)) * nu;
                T ref[5];
#pragma unroll
                for (int vv = 0; vv < 5; ++vv) ref[vv] = avg_right(qR[vv], dq[vv], q6[vv], y);
                T bz = T(0), bm = T(0);
                if (l0 > T(0)) {
                    T y0 = l0 * nu;
                    bz = (ref[0] - avg_right(qR[0], dq[0], q6[0], y0)) - (ref[4] - avg_right(qR[4], dq[4], q6[4], y0)) * ic2;
                }
                if (lm > T(0)) {
                    T ym = lm * nu;
                    T du = ref[1] - avg_right(qR[1], dq[1], q6[1], ym);
                    T dp = ref[4] - avg_right(qR[4], dq[4], q6[4], ym);
                    bm = dp * i2c2 - rc2 * du;
                }
                T yv = tmax(l0, T(0)) * nu;
                TL.r = ref[0] - bz - bm;
                TL.u = ref[1] + bm * cr_;
                TL.v = avg_right(qR[2], dq[2], q6[2], yv);
                TL.w = avg_right(qR[3], dq[3], q6[3], yv);
                TL.p = ref[4] - bm * c2;
            }
            {   // left face: waves moving left
                T y = tmax(-lm, T(0)) * nu;
                T ref[5];
#pragma unroll
                for (int vv = 0; vv < 5; ++vv) ref[vv] = avg_left(qL[vv], dq[vv], q6[vv], y);
                T bz = T(0), bp = T(0);
                if (l0 < T(0)) {
                    T y0 = -l0 * nu;
                    bz = (ref[0] - avg_left(qL[0], dq[0], q6[0], y0)) - (ref[4] - avg_left(qL[4], dq[4], q6[4], y0)) * ic2;
                }
                if (lp < T(0)) {
                    T yp = -lp * nu;
                    T du = ref[1] - avg_left(qL[1], dq[1], q6[1], yp);
                    T dp = ref[4] - avg_left(qL[4], dq[4], q6[4], yp);
                    bp = dp * i2c2 + rc2 * du;
                }
                T yv = tmax(-l0, T(0)) * nu;
                TR.r = ref[0] - bz - bp;
                TR.u = ref[1] - bp * cr_;
                TR.v = avg_left(qL[2], dq[2], q6[2], yv);
                TR.w = avg_left(qL[3], dq[3], q6[3], yv);
                TR.p = ref[4] - bp * c2;
            }
            // half-step sources: gravity on rho' (momentum), base advection
            T su = hdt * (q[2][0] * gr[1] / rj);
            T sr = hdt * (uj * (r0f[1] - r0f[0]) * rdx);
            T sp = hdt * (uj * (p0f[1] - p0f[0]) * rdx);
            TL.u += su; TR.u += su;
            TL.r -= sr; TR.r -= sr;
            TL.p -= sp; TR.p -= sp;
        }
        // ---- (5) Riemann problem and fluxes at face (k-3)+1/2
        T F[5] = { T(0), T(0), T(0), T(0), T(0) };
        T sg = T(0);
        if (k >= 1) {
            St<T> Ls = TLp, Rs = TR;
            const bool sa = sol[1], sb = sol[2];
            if (sa && sb) {
                for (int vv = 0; vv < 5; ++vv) F[vv] = T(0);
            } else {
                if (sb) { Rs = Ls; Rs.u = -Ls.u; }          // wall: mirror the fluid side (Sec. 3)
                if (sa) { Ls = Rs; Ls.u = -Rs.u; }
                bool cnt;
                St<T> f = Solver<T>::solve(Ls, Rs, r0f[0], p0f[0], gam, cnt);
                if (cnt && k - 3 >= -1 && k - 3 < n) ++c_rie;
                T rf = r0f[0] + f.r;
                T Fr = rf * f.u;
                F[0] = Fr;
                F[1] = Fr * f.u + f.p;
                F[2] = Fr * f.v;
                F[3] = Fr * f.w;
                F[4] = f.u * (gfac * (p0f[0] + f.p) + T(0.5) * rf * ((f.u * f.u + f.v * f.v) + f.w * f.w));
                sg = f.u * nu;
            }
        }
        TLp = TL;
        // ---- (6) conservative update of cell k-3 (written one step later)
        T hn[5] = { T(0), T(0), T(0), T(0), T(0) };
        const int cu_ = k - 3;
        if (cu_ >= 0 && cu_ < n) {
            if (sol[1]) {
                for (int vv = 0; vv < 5; ++vv) hn[vv] = cu[0][vv];
            } else {
                T rn = cu[0][0] - nu * (F[0] - Fp[0]);
                hn[0] = rn;
                hn[1] = cu[0][1] - nu * (F[1] - Fp[1]) + dt * gr[0] * (T(0.5) * (cu[0][0] + rn));
                hn[2] = cu[0][2] - nu * (F[2] - Fp[2]);
                hn[3] = cu[0][3] - nu * (F[3] - Fp[3]);
                hn[4] = cu[0][4] - nu * (F[4] - Fp[4]) + dt * gr[0] * (T(0.5) * (Fp[0] + F[0]));
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
                if (sg1 > T(0)) {
                    slab(pqp, sg1, Lp, G);
                } else if (sg1 < T(0)) {
                    T fq[10];
#pragma unroll
                    for (int v = 0; v < 10; ++v) fq[v] = (v == 1 || v == 4 || v == 6) ? -pql[v] : pql[v];
                    slab(fq, sg1, Ld, G);
                } else {
#pragma unroll
                    for (int v = 0; v < 10; ++v) G[v] = T(0);
                }
                const int cw = k - 4;
                if (cw >= 0 && cw < n) {
                    long ci = base + cw * sAX;
                    T o[10];
                    double xs[3] = { xt[0], xt[1], xt[2] };
                    xs[AX] = centre(g, AX, cw);
                    const bool solid_w = sol[0];
                    if (solid_w) {
#pragma unroll
                        for (int v = 0; v < 10; ++v) o[v] = in[AI::ppb(v) * nc + ci];
                    } else {
                        ppb_update(pqp, sg1 - sg2, T(0.5) * (sg2 + sg1), Gp, G, o);
                    }
                    T e = hyd[4];
                    if (a.heat && !solid_w) e = T((double)e + heating(g, xs[0], xs[1], xs[2]) * dt64);
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

template <typename T, int AX>
__global__ __launch_bounds__(64)
void sweep_kernel(Geom g, SweepArgs<T> a)
{
    // lanes run across x for the y and z passes, across y for the x pass
    const int ca = (AX == 0) ? 1 : 0;
    const int cb = 3 - AX - ca;
    const int nblk_a = (g.n[ca] + 63) / 64;
    const int la = (blockIdx.x % nblk_a) * 64 + threadIdx.x;
    const int lb = blockIdx.x / nblk_a;
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

template <typename T>
hipError_t launch_sweep(const Geom &g, int axis, const T *in, T *out, const T *rho0, const T *p0,
                        const double *dtp, unsigned long long *counters, int heat, hipStream_t st)
{
    SweepArgs<T> a{in, out, rho0, p0, dtp, counters, (long)g.n[0] * g.n[1] * g.n[2], heat};
    const int ca = (axis == 0) ? 1 : 0;
    const int cb = 3 - axis - ca;
    const long nblk = (long)((g.n[ca] + 63) / 64) * g.n[cb];
    if (nblk <= 0 || nblk > 0x7fffffffL) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblk), block(64);
    switch (axis) {
    case 0: hipLaunchKernelGGL((sweep_kernel<T, 0>), grid, block, 0, st, g, a); break;
    case 1: hipLaunchKernelGGL((sweep_kernel<T, 1>), grid, block, 0, st, g, a); break;
    default: hipLaunchKernelGGL((sweep_kernel<T, 2>), grid, block, 0, st, g, a); break;
    }
    return hipGetLastError();
}

template hipError_t launch_sweep<float>(const Geom &, int, const float *, float *, const float *,
                                        const float *, const double *, unsigned long long *, int,
                                        hipStream_t);
template hipError_t launch_sweep<double>(const Geom &, int, const double *, double *,
                                         const double *, const double *, const double *,
                                         unsigned long long *, int, hipStream_t);

}  // namespace ppmb
