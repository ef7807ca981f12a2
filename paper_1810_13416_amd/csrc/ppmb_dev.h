// ppmb_dev.h -- device building blocks of the 1-D PPM + PPB pass (gfx950).
//
// Each function is one step of the pass as the paper describes it in words
// (Sec. 1, Sec. 4), with the formulas of the canonical PPM paper (Colella &
// Woodward 1984, "CW84") where the paper defers to its references.  All are
// templated on the working precision T (float or double).
#pragma once
#include <hip/hip_runtime.h>

namespace ppmb {

enum { NG = 4, NF = 15 };
enum { RHO = 0, MX = 1, MY = 2, MZ = 3, EN = 4, F0 = 5, FX = 6, FY = 7, FZ = 8,
       FXX = 9, FYY = 10, FZZ = 11, FXY = 12, FYZ = 13, FZX = 14 };

// Grid and physics parameters, passed by value to every kernel.
struct Geom {
    int    n[3];
    double dx;
    double origin[3];
    int    bc[3];
    double gamma;
    int    sphere;
    double sphere_r;
    double sphere_t;      // least r^2 whose correctly rounded sqrt is >= sphere_r
    int    grav_kind;
    double grav[4];
    int    heat_kind;
    double heat[3];
    int    smooth_detect;
    // The pass kernels' gravity and heating constants in both working
    // precisions, derived once on the host (each the FP64 value rounded):
    // gravity kind 1: gx, gy, gz; kind 2: g0, rc, 1/rc, r1, r2, 1/(r2 - r1);
    // heating: Q0, 1/extent, z0.
    float  gcf[6];
    double gcd[6];
    float  hcf[3];
    double hcd[3];
    // storage: cell (i, j, k) of field q at q * fs + i + j * px + k * plane
    // (rows start on 256-byte boundaries; fs is padded so that the fields do
    // not all fall on the same cache sets)
    int    px;
    long   plane;
    long   fs;
};

// Storage offset of the cell with dense (x fastest) number c.
__host__ __device__ __forceinline__ long pitched(const Geom &g, long c)
{
    const unsigned nx = (unsigned)g.n[0], ny = (unsigned)g.n[1];
    const unsigned cc = (unsigned)c;                 // bricks hold fewer than 2^32 cells
    const unsigned row = cc / nx, i = cc - row * nx;
    const unsigned k = row / ny, j = row - k * ny;
    return (long)i + (long)j * g.px + (long)k * g.plane;
}

// Reciprocal, reciprocal square root and square root.  FP32: the hardware
// instructions (1 ulp), without the denormal rescaling the compiler wraps
// around them: no quantity of the pass comes near the FP32 denormal range
// (densities, pressures and sound speeds are O(1e-3 .. 1e3)).  FP64:
// correctly rounded.
__device__ __forceinline__ float trcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ double trcp(double a) { return 1.0 / a; }
__device__ __forceinline__ float trsq(float a) { return __builtin_amdgcn_rsqf(a); }
__device__ __forceinline__ double trsq(double a) { return 1.0 / sqrt(a); }
__device__ __forceinline__ float tsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double tsqrt(double a) { return sqrt(a); }

// Sound speed c = sqrt(x) and 1/c of x = gamma p / rho, from one
// reciprocal square root.
template <typename T>
__device__ __forceinline__ void sound(T x, T &c, T &ic)
{
    ic = trsq(x);
    c = x * ic;
}

// hardware abs / min / max (operand modifiers and single instructions)
__device__ __forceinline__ float tabs(float a) { return fabsf(a); }
__device__ __forceinline__ double tabs(double a) { return fabs(a); }
__device__ __forceinline__ float tmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double tmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float tmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double tmax(double a, double b) { return fmax(a, b); }

// ---------------------------------------------------------------------
// Geometry: ghost mapping, gravity, heating, confining sphere
// ---------------------------------------------------------------------

// Source cell of pencil index j on an axis of n cells; flip = -1 when the
// cell is seen through an odd number of reflecting walls.
__device__ __forceinline__ int bc_source(int j, int n, int bc, int &flip)
{
    flip = 1;
    if (bc == 0) {
        int k = j % n;
        return k < 0 ? k + n : k;
    }
    int p = 2 * n;
    int k = j % p;
    if (k < 0) k += p;
    if (k < n) return k;
    flip = -1;
    return p - 1 - k;
}

// Cell-centre coordinate (FP64).
__device__ __forceinline__ double centre(const Geom &g, int axis, int i)
{
    // rounded product, then rounded sum, in every unit whatever its
    // contraction setting: the same number as on the host
    return __dadd_rn(g.origin[axis], __dmul_rn((double)i + 0.5, g.dx));
}

// |x|^2 evaluated without contraction so that the solid test agrees
// bit for bit with any IEEE implementation of the same expression.
__device__ __forceinline__ double r2_exact(double x, double y, double z)
{
    return __dadd_rn(__dadd_rn(__dmul_rn(x, x), __dmul_rn(y, y)), __dmul_rn(z, z));
}

// Sec. 3: cells outside the inscribed sphere are solid: sqrt(|x|^2) >= R.
// The square root is correctly rounded and monotone, so the test is the
// same as |x|^2 >= sphere_t, the threshold the host finds once.
__device__ __forceinline__ bool solid_at(const Geom &g, double x, double y, double z)
{
    if (!g.sphere) return false;
    return r2_exact(x, y, z) >= g.sphere_t;
}

// Sec. 3: gravity falls to zero a few cells before the sphere; linear taper.
__device__ __forceinline__ double grav_taper(const Geom &g, double r)
{
    if (r <= g.grav[2]) return 1.0;
    if (r >= g.grav[3]) return 0.0;
    return (g.grav[3] - r) / (g.grav[3] - g.grav[2]);
}

// Component `axis` of the gravitational acceleration at a point, in the
// working precision; rt2 is the squared distance to the centre; c the
// grid's constants in that precision (gcf / gcd of Geom).
template <typename T, typename C>
__device__ __forceinline__ T gravity(int kind, const C *c, int axis, T xd, T rt2)
{
    // every constant is read before any branch, so that the loads are
    // issued together and waited for once
    const T c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5];
    if (kind == 1) return axis == 0 ? c0 : (axis == 1 ? c1 : c2);
    if (kind == 2) {
        // r and 1/r^3 from one reciprocal square root (r = 0 at the centre)
        const T ir = trsq(rt2);
        const T r = rt2 > T(0) ? rt2 * ir : T(0);
        T h = (r < c1) ? c2 : (c1 * c1) * (ir * ir * ir);
        T t = r <= c3 ? T(1) : (r >= c4 ? T(0) : (c4 - r) * c5);
        return -c0 * xd * h * t;
    }
    return T(0);
}

// Heating profile: full below half the extent, smoothstep to zero at it.
template <typename T>
__device__ __forceinline__ T heat_shape(T xi)
{
    if (xi <= T(0.5)) return T(1);
    if (xi >= T(1)) return T(0);
    T t = T(2) * xi - T(1);
    return T(1) - t * t * (T(3) - T(2) * t);
}

// c: the grid's heating constants in the working precision (hcf / hcd).
template <typename T, typename C>
__device__ __forceinline__ T heating(int kind, const C *c, T z, T rt2)
{
    const T c0 = c[0], c1 = c[1], c2 = c[2];       // read before any branch, as in gravity
    if (kind == 1) return c0 * heat_shape((z - c2) * c1);
    if (kind == 2) return c0 * heat_shape(tsqrt(rt2) * c1);
    return T(0);
}

// Fluid cells of a pencil along `axis` through the cell centres with
// transverse coordinates fixed: the exact solid test is monotone in the
// distance from the pencil's closest point to the centre, so the fluid
// cells form one interval [lo, hi] (empty: lo > hi), found by bisection
// with the same FP64 test as everywhere else.
__device__ __forceinline__ void fluid_interval(const Geom &g, int axis, const double xt[3], int &lo, int &hi)
{
    const int n = g.n[axis];
    lo = 0;
    hi = n - 1;
    if (!g.sphere) return;
    auto solid = [&](int i) {
        double x[3] = { xt[0], xt[1], xt[2] };
        x[axis] = centre(g, axis, i);
        return solid_at(g, x[0], x[1], x[2]);
    };
    // index nearest to coordinate 0 along the pencil, and its neighbours
    double fm = -g.origin[axis] / g.dx - 0.5;
    int m = (int)floor(fm + 0.5);
    m = m < 0 ? 0 : (m > n - 1 ? n - 1 : m);
    int best = -1;
    for (int c = m - 1; c <= m + 1; ++c)
        if (c >= 0 && c < n && !solid(c)) { best = c; break; }
    if (best < 0) { lo = 1; hi = 0; return; }
    int a = 0, b = best;                 // first fluid index in [0, best]
    while (a < b) { int mid = (a + b) / 2; if (solid(mid)) a = mid + 1; else b = mid; }
    lo = a;
    a = best; b = n - 1;                 // last fluid index in [best, n-1]
    while (a < b) { int mid = (a + b + 1) / 2; if (solid(mid)) b = mid - 1; else a = mid; }
    hi = a;
}

// Largest signal speed max_d |u_d| + c of one cell from its stored
// conserved perturbations and FP64 base, in FP64 without contraction, so
// that it is the same number wherever it is evaluated (the CFL kernel and
// the last pass of a step).  `bad`: non-positive density or pressure, NaN
// or overflow.
__device__ __forceinline__ double cell_speed(double r0, double p0, double rp, double mx, double my,
                                             double mz, double ep, double gamma, bool &bad)
{
#pragma clang fp contract(off)
    const double gm1 = gamma - 1.0;
    const double rho = r0 + rp;
    const double u = mx / rho, v = my / rho, w = mz / rho;
    const double pp = gm1 * (ep - 0.5 * (mx * u + my * v + mz * w));
    const double p = p0 + pp;
    const double cs = sqrt(gamma * p / rho);
    const double sp = fmax(fabs(u), fmax(fabs(v), fabs(w))) + cs;
    bad = !(rho > 0.0) || !(p > 0.0) || !(sp == sp) || sp > 1e300;
    return sp;
}

// Whether a cell's signal speed can reach `thr`, from the working-precision
// values the pass holds: an upper bound of cell_speed (base from the
// working-precision copy, rounding of every operation covered a hundred
// times over by the 1e-5 margins) compared with thr.  A cell whose density
// is not clearly positive or whose pressure bound is not positive always
// answers yes, so that cell_speed sees every possibly non-physical cell.
template <typename T>
__device__ __forceinline__ bool speed_may_reach(T r0, T p0, T rp, T m1, T m2, T m3, T ep, T gam, T gm1, T thr)
{
    const T rho = r0 + rp;
    if (!(rho > T(0.5) * r0) || !(rho > T(0))) return true;
    const T ir = trcp(rho);
    const T ke2 = (m1 * m1 + m2 * m2 + m3 * m3) * ir;
    const T p = p0 + gm1 * (ep - T(0.5) * ke2);
    const T err = T(1e-5) * (tabs(p0) + gm1 * (tabs(ep) + T(0.5) * ke2));
    if (!(p - err > T(0))) return true;
    const T umax = tmax(tabs(m1), tmax(tabs(m2), tabs(m3))) * ir;
    const T s = (umax + tsqrt(gam * (p + err) * ir)) * T(1.00001);
    return !(s < thr);
}

// ---------------------------------------------------------------------
// PPM reconstruction (Sec. 1)
// ---------------------------------------------------------------------

// Interface value one order higher than the parabola: the 4th-order value
// from the four cell averages around the face (CW84 eq. 1.6, uniform grid).
template <typename T>
__device__ __forceinline__ T face4(T am, T a, T b, T bp)
{
    return (T(7) * (a + b) - (am + bp)) * T(1.0 / 12.0);
}

// 5-cell smoothness judgment (Sec. 1), graded: weight 1 (no constraints)
// when the three second differences in the window are all zero, or share
// one strict sign with max <= 2 min in magnitude; weight 0 when their signs
// differ or max >= 3 min; linear in between, so that the reconstruction
// depends continuously on the data.  Returns the weight of the
// unconstrained parabola.
template <typename T>
__device__ __forceinline__ T smooth_weight(T q0, T q1, T q2, T q3, T q4)
{
    T d0 = (q0 + q2) - T(2) * q1;
    T d1 = (q1 + q3) - T(2) * q2;
    T d2 = (q2 + q4) - T(2) * q3;
    if (d0 == T(0) && d1 == T(0) && d2 == T(0)) return T(1);
    bool same = (d0 > T(0) && d1 > T(0) && d2 > T(0)) || (d0 < T(0) && d1 < T(0) && d2 < T(0));
    if (!same) return T(0);
    T a0 = tabs(d0), a1 = tabs(d1), a2 = tabs(d2);
    T mx = tmax(a0, tmax(a1, a2)), mn = tmin(a0, tmin(a1, a2));
    if (mx <= T(2) * mn) return T(1);
    if (mx >= T(3) * mn) return T(0);
    return (T(3) * mn - mx) * trcp(mn);
}

// The same judgment from the three second differences themselves.
template <typename T>
__device__ __forceinline__ T smooth_weight_d(T d0, T d1, T d2)
{
    // one strict sign <=> the smallest is > 0 or the largest is < 0
    const T lo = tmin(d0, tmin(d1, d2)), hi = tmax(d0, tmax(d1, d2));
    const T a0 = tabs(d0), a1 = tabs(d1), a2 = tabs(d2);
    const T mx = tmax(a0, tmax(a1, a2)), mn = tmin(a0, tmin(a1, a2));
    const bool below = mx <= T(2) * mn, above = mx >= T(3) * mn;
    T w = below ? T(1) : T(0);
    // the graded band between: few cells of a wave lie in it, so the
    // reciprocal is computed only when one does
    const bool band = !below && !above;
    if (__builtin_amdgcn_ballot_w64(band)) {
        const T r = (T(3) * mn - mx) * trcp(mn);
        w = band ? r : w;
    }
    w = (lo > T(0) || hi < T(0)) ? w : T(0);
    return mx == T(0) ? T(1) : w;
}

// van Leer limited slope (CW84 eq. 1.8).
template <typename T>
__device__ __forceinline__ T limited_slope(T qm, T q, T qp)
{
    T dl = q - qm, dr = qp - q;
    T dc = T(0.5) * (qp - qm);
    T m = tmin(tabs(dc), tmin(T(2) * tabs(dl), T(2) * tabs(dr)));
    m = dc > T(0) ? m : -m;
    return (dl * dr > T(0)) ? m : T(0);
}

// Face value from limited slopes, symmetric in the two cells at the face.
template <typename T>
__device__ __forceinline__ T face_limited(T qa, T qb, T sa, T sb)
{
    return T(0.5) * (qa + qb) - (sb - sa) * T(1.0 / 6.0);
}

// CW84 eq. 1.10: extremum and overshoot constraints on the edge values.
// Branch-free: in a wave some cell nearly always takes each path, so
// selects cost less than divergent branches.
template <typename T>
__device__ __forceinline__ void constrain(T q, T &qL, T &qR)
{
    // a local extremum flattens the cell; else an overshoot on one side
    // moves that edge (the left test first)
    const bool ext = (qR - q) * (q - qL) <= T(0);
    const T dq = qR - qL;
    const T q6 = T(6) * (q - T(0.5) * (qL + qR));
    const bool ovl = dq * q6 > dq * dq;
    const bool ovr = !ovl && dq * q6 < -(dq * dq);
    const T nl = ext ? q : (ovl ? T(3) * q - T(2) * qR : qL);
    const T nr = ext ? q : (ovr ? T(3) * q - T(2) * qL : qR);
    qL = nl;
    qR = nr;
}

// Averages of the parabola over the last / first fraction y of the cell.
template <typename T>
__device__ __forceinline__ T avg_right(T qR, T dq, T q6, T y)
{
    return qR - (T(0.5) * y) * (dq - (T(1) - T(2.0 / 3.0) * y) * q6);
}
template <typename T>
__device__ __forceinline__ T avg_left(T qL, T dq, T q6, T y)
{
    return qL + (T(0.5) * y) * (dq + (T(1) - T(2.0 / 3.0) * y) * q6);
}

// ---------------------------------------------------------------------
// Riemann solver on the pressure perturbation (CW84 Sec. 2)
// ---------------------------------------------------------------------

// State at a face: rho', u, v, w, p'.
template <typename T> struct St { T r, u, v, w, p; };

// Newton iterations of the two-shock approximation.  p0f cancels from every
// pressure difference; the full pressures only set the wave impedances.
// Written with reciprocals: 1/W from one rsqrt per side, the linearised
// impedances as 1/Z = (1 + C^2 / W^2) / (2 W), so that an iteration costs
// two rsqrt and one reciprocal.  Stops once the pre-update velocity residual
// |u*_R - u*_L| is at most tol (cL + cR); returns whether that happened
// within `maxit` iterations.  Outputs p'*, u*, 1/W_L, 1/W_R.
template <typename T>
struct Face {
    T rL, rR, irL, irR;   // full densities and their reciprocals
    T pL, pR, ipL, ipR;   // full pressures and their reciprocals
    T CL, CR, iCL, iCR;   // Lagrangian sound speeds sqrt(gamma p rho) and reciprocals
};

template <typename T>
__device__ __forceinline__ Face<T> face_setup(const St<T> &L, const St<T> &R, T r0f, T p0f, T gamma)
{
    Face<T> F;
    F.rL = r0f + L.r;
    F.rR = r0f + R.r;
    F.pL = p0f + L.p;
    F.pR = p0f + R.p;
    F.irL = trcp(F.rL);
    F.irR = trcp(F.rR);
    F.ipL = trcp(F.pL);
    F.ipR = trcp(F.pR);
    T gL = gamma * F.pL * F.rL, gR = gamma * F.pR * F.rR;
    F.iCL = trsq(gL);
    F.iCR = trsq(gR);
    F.CL = gL * F.iCL;
    F.CR = gR * F.iCR;
    return F;
}

template <typename T>
__device__ __forceinline__ bool two_shock(const St<T> &L, const St<T> &R, const Face<T> &F, T p0f,
                                          T gamma, int maxit, T tol, T &ps, T &us, T &iWL, T &iWR)
{
    const T A = (gamma + T(1)) * trcp(T(2) * gamma);
    const T cs = F.CL * F.irL + F.CR * F.irR;
    const T pfl = T(1e-10) * tmin(F.pL, F.pR) - p0f;
    ps = (F.CR * L.p + F.CL * R.p + F.CL * F.CR * (L.u - R.u)) * trcp(F.CL + F.CR);
    if (ps < pfl) ps = pfl;
    iWL = F.iCL;
    iWR = F.iCR;
    us = T(0.5) * (L.u + R.u);
    const T CL2 = F.CL * F.CL, CR2 = F.CR * F.CR;
    // Newton steps until the velocity residual at the current p* is within
    // tol (cL + cR); the step taken with it is kept.  A wave leaves the
    // loop when all its lanes have: at low Mach numbers the acoustic guess
    // already passes, after one step
    for (int it = 0; it < maxit; ++it) {
        iWL = F.iCL * trsq(T(1) + A * (ps - L.p) * F.ipL);
        iWR = F.iCR * trsq(T(1) + A * (ps - R.p) * F.ipR);
        T uLs = L.u - (ps - L.p) * iWL;
        T uRs = R.u + (ps - R.p) * iWR;
        T iZL = T(0.5) * iWL * (T(1) + CL2 * iWL * iWL);
        T iZR = T(0.5) * iWR * (T(1) + CR2 * iWR * iWR);
        T rden = trcp(iZL + iZR);
        T du = uRs - uLs;
        us = (uLs * iZR + uRs * iZL) * rden;
        ps = ps - du * rden;
        if (ps < pfl) ps = pfl;
        if (tabs(du) <= tol * cs) return true;
    }
    return false;
}

// Sample the face state by the sign of u* and the speed of the wave on
// that side (CW84 Sec. 2); the side is unshocked when that wave has
// already passed the face: u_s -+ W_s / rho_s of the sign of u*.
template <typename T>
__device__ __forceinline__ St<T> sample(const St<T> &L, const St<T> &R, const Face<T> &F, T ps, T us,
                                        T iWL, T iWR)
{
    // field-wise selects (no selection between whole structs, which would
    // put the states in scratch memory)
    const bool lft = us >= T(0);
    const T r = lft ? L.r : R.r, u = lft ? L.u : R.u, v = lft ? L.v : R.v;
    const T w = lft ? L.w : R.w, p = lft ? L.p : R.p;
    const T rr = lft ? F.rL : F.rR, iW = lft ? iWL : iWR;
    const T su = lft ? u : -u;
    St<T> f;
    if (su * rr * iW >= T(1)) {                  // the wave has passed the face
        f.r = r; f.u = u; f.v = v; f.w = w; f.p = p;
    } else {
        T X = rr * (ps - p) * (iW * iW);
        f.r = r + rr * X * trcp(T(1) - X);
        f.u = us; f.v = v; f.w = w; f.p = ps;
    }
    return f;
}

// Full solve.  FP64: Newton to a velocity residual of 1e-13 (cL + cR), at
// most 20 iterations.  FP32: two iterations, then, if the residual is still
// above 1e-5, the FP64 solve from the same states (counted in `refined`).
__device__ __forceinline__ St<double> riemann64(const St<double> &L, const St<double> &R,
                                                double r0f, double p0f, double gamma, bool &bad)
{
    Face<double> F = face_setup<double>(L, R, r0f, p0f, gamma);
    double ps, us, iWL, iWR;
    bad = !two_shock<double>(L, R, F, p0f, gamma, 20, 1e-13, ps, us, iWL, iWR);
    return sample<double>(L, R, F, ps, us, iWL, iWR);
}

template <typename T> struct Solver;

template <> struct Solver<double> {
    __device__ static St<double> solve(const St<double> &L, const St<double> &R, double r0f,
                                       double p0f, double gamma, bool &counted)
    {
        return riemann64(L, R, r0f, p0f, gamma, counted);
    }
};

template <> struct Solver<float> {
    __device__ static St<float> solve(const St<float> &L, const St<float> &R, float r0f,
                                      float p0f, float gamma, bool &counted)
    {
        Face<float> F = face_setup<float>(L, R, r0f, p0f, gamma);
        float ps, us, iWL, iWR;
        bool ok = two_shock<float>(L, R, F, p0f, gamma, 2, 1e-5f, ps, us, iWL, iWR);
        counted = false;
        if (!ok) {
            counted = true;
            St<double> Ld{L.r, L.u, L.v, L.w, L.p}, Rd{R.r, R.u, R.v, R.w, R.p};
            bool bad;
            St<double> f = riemann64(Ld, Rd, (double)r0f, (double)p0f, (double)gamma, bad);
            return St<float>{(float)f.r, (float)f.u, (float)f.v, (float)f.w, (float)f.p};
        }
        return sample<float>(L, R, F, ps, us, iWL, iWR);
    }
};

// ---------------------------------------------------------------------
// PPB (Sec. 1, Sec. 4): Lagrange-remap transport of fv and its moments
// ---------------------------------------------------------------------

// Constraint applied almost never (Sec. 1): scale the slope and curvature
// along the pass so that a0 + a1 s + a2 (s^2 - 1/12) stays in [0, 1] on the
// cell.  Returns true when the profile changed by more than round-off.
template <typename T>
__device__ __forceinline__ bool fv_limit(T a0, T &a1, T &a2)
{
    // Quick acceptance: on the cell |a1 s| <= |a1|/2 and |a2 (s^2 - 1/12)|
    // <= |a2|/6, so a profile whose bound a0 -+ e lies inside [0, 1] by more
    // than the rounding of the exact test below is left as it is, exactly
    // as the exact test would leave it.
    {
        const T eps = sizeof(T) == 4 ? T(1.0 / 16777216.0) : T(1.0 / 9007199254740992.0);
        const T e = T(0.5) * tabs(a1) + tabs(a2) * T(1.0 / 6.0);
        const T m = T(16) * eps * (tabs(a0) + tabs(a1) + tabs(a2));
        if (a0 - e >= m && a0 + e <= T(1) - m) return false;
    }
    T gm = a0 - T(0.5) * a1 + a2 * T(1.0 / 6.0);
    T gp = a0 + T(0.5) * a1 + a2 * T(1.0 / 6.0);
    T lo = tmin(gm, gp), hi = tmax(gm, gp);
    if (tabs(a1) < tabs(a2)) {                 // vertex -a1 / (2 a2) inside the cell
        T gv = a0 - a2 * T(1.0 / 12.0) - (a1 * a1) * trcp(T(4) * a2);
        lo = tmin(lo, gv);
        hi = tmax(hi, gv);
    }
    if (!(hi > T(1) || lo < T(0))) return false;
    T th = T(1);
    if (hi > T(1)) th = tmin(th, (T(1) - a0) / (hi - a0));
    if (lo < T(0)) th = tmin(th, a0 / (a0 - lo));
    if (!(th < T(1))) return false;
    if (th < T(0)) th = T(0);
    T s1 = tabs(a1) + tabs(a2);
    a1 *= th;
    a2 *= th;
    return (T(1) - th) * s1 > T(1e-9);
}

// Pass-local fv coefficients: q[0..2] quadratic along the pass, q[3..4] and
// q[5..6] transverse slopes varying linearly along it, q[7..9] constants.
struct PPBIdx { int f[10]; };

// Moments about the face of the donor slab crossing it.  sig = u* dt/dx at
// the face; the donor has Lagrangian length L and coefficients q (odd-in-s
// entries flipped by the caller for a donor on the right).  Slab integrals
// over s = 1/2 - t + t u, u in [0, 1], t = |sig| / L.
template <typename T>
__device__ __forceinline__ void slab(const T *q, T sig, T L, T *G)
{
    T t = tabs(sig) * trcp(L);
    T h = T(0.5) - t;
    T al0 = q[0] + q[1] * h + q[2] * (h * h - T(1.0 / 12.0));
    T al1 = t * (q[1] + T(2) * q[2] * h);
    T al2 = q[2] * (t * t);
    T I0 = al0 + al1 * T(0.5) + al2 * T(1.0 / 3.0);
    T I1 = al0 * T(0.5) + al1 * T(1.0 / 3.0) + al2 * T(0.25);
    T I2 = al0 * T(1.0 / 3.0) + al1 * T(0.25) + al2 * T(0.2);
    T s2 = sig * sig, s3 = s2 * sig;
    G[0] = sig * I0;
    G[1] = s2 * I1;
    G[2] = s3 * I2;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        T b0 = q[3 + 2 * p], b1 = q[4 + 2 * p];
        T be0 = b0 + b1 * h;
        T be1 = b1 * t;
        G[3 + 2 * p] = sig * (be0 + be1 * T(0.5));
        G[4 + 2 * p] = s2 * (be0 * T(0.5) + be1 * T(1.0 / 3.0));
    }
    G[7] = sig * q[7];
    G[8] = sig * q[8];
    G[9] = sig * q[9];
}

// New coefficients of a cell: its Lagrangian content about the cell centre
// (length L, centre offset dl, stretch ds = L - 1) minus the slab leaving
// through the right face (GR) plus the one entering through the left (GL),
// both shifted from the face to the centre.
template <typename T>
__device__ __forceinline__ void ppb_update(const T *q, T ds, T dl, const T *GL, const T *GR, T *o)
{
    T L = T(1) + ds;
    T a0 = q[0], a1 = q[1], a2 = q[2];
    T M0 = L * a0;
    T M1 = L * (dl * a0 + L * a1 * T(1.0 / 12.0));
    T M2 = L * (dl * dl * a0 + dl * L * a1 * T(1.0 / 6.0) + L * L * a2 * T(1.0 / 180.0)
                + a0 * ds * (T(2) + ds) * T(1.0 / 12.0));
    o[0] = M0 - (GR[0] - GL[0]);
    o[1] = T(12) * (M1 - (GR[1] - GL[1]) - T(0.5) * (GR[0] + GL[0]));
    o[2] = T(180) * (M2 - (GR[2] - GL[2]) - (GR[1] + GL[1]) - (GR[0] - GL[0]) * T(1.0 / 6.0));
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        int b = 3 + 2 * p;
        T b0 = q[b], b1 = q[b + 1];
        T N0 = L * b0;
        T N1 = L * (dl * b0 + L * b1 * T(1.0 / 12.0));
        o[b] = N0 - (GR[b] - GL[b]);
        o[b + 1] = T(12) * (N1 - (GR[b + 1] - GL[b + 1]) - T(0.5) * (GR[b] + GL[b]));
    }
#pragma unroll
    for (int c = 7; c < 10; ++c) o[c] = L * q[c] - (GR[c] - GL[c]);
}

// ---------------------------------------------------------------------
// Per-cell and per-face stages of the pass, shared by both kernel shapes
// ---------------------------------------------------------------------

// Edge values of one variable's parabola in cell q: the unconstrained
// 4th-order face values (qfL, qfR) unless the 5-cell judgment (second
// differences d0..d2) says otherwise, then the CW84-constrained values from
// the limited-slope faces (flL, flR), blended over the graded band.
// Returns true when constraints entered.
template <typename T>
__device__ __forceinline__ bool parabola(int detect, T q, T qfL, T qfR, T flL, T flR, T d0, T d1, T d2,
                                         T &l, T &r)
{
    // branch-free: in a wave some cell is nearly always constrained
    const T ws = detect == 1 ? smooth_weight_d(d0, d1, d2) : T(detect == 2 ? 1 : 0);
    T lc = flL, rc = flR;
    constrain(q, lc, rc);
    const bool con = ws < T(1);
    const bool blend = ws > T(0);
    const T lb = lc + ws * (qfL - lc), rb = rc + ws * (qfR - rc);
    l = con ? (blend ? lb : lc) : qfL;
    r = con ? (blend ? rb : rc) : qfR;
    return con;
}

// Characteristic tracing of one cell (CW84 Sec. 3): the states at its right
// face (TL, seen from the left of that face) and at its left face (TR), from
// the parabolas of rho', u, v, w, p' (edge values qL, qR, dq, q6), the
// cell's rho and 1/rho, c and 1/c, u, rho', gravity, and the base face
// values, plus the half-step sources (gravity on rho', advection of the
// base).
template <typename T>
__device__ __forceinline__ void trace_cell(const T *qL, const T *qR, const T *dq, const T *q6,
                                           T rj, T irj, T cj, T icj, T uj, T rpj, T gj, T r0fL, T r0fR,
                                           T p0fL, T p0fR, T nu, T hdt, T rdx, St<T> &TL, St<T> &TR)
{
    const T c2 = cj * cj;
    const T lm = uj - cj, l0 = uj, lp = uj + cj;
    const T rc2 = T(0.5) * rj * icj, cr_ = cj * irj, ic2 = icj * icj, i2c2 = T(0.5) * ic2;
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
    T su = hdt * (rpj * gj * irj);
    T sr = hdt * (uj * (r0fR - r0fL) * rdx);
    T sp = hdt * (uj * (p0fR - p0fL) * rdx);
    TL.u += su; TR.u += su;
    TL.r -= sr; TR.r -= sr;
    TL.p -= sp; TR.p -= sp;
}

// Riemann problem and fluxes at one face (states Ls | Rs; sa, sb: the two
// cells are solid).  A face between a fluid and a solid cell is a
// reflecting wall (Sec. 3): the solid side takes the mirrored fluid state.
// F = mass, normal, two transverse momenta, energy; sg = u* dt/dx.
// Returns true when the Riemann problem was counted (FP64 re-solve).
template <typename T>
__device__ __forceinline__ bool face_flux(St<T> Ls, St<T> Rs, bool sa, bool sb, T r0f, T p0f, T gam,
                                          T gfac, T nu, T *F, T &sg)
{
    if (sa && sb) {
#pragma unroll
        for (int vv = 0; vv < 5; ++vv) F[vv] = T(0);
        sg = T(0);
        return false;
    }
    // a wall mirrors the fluid side (sa and sb exclusive here); field-wise
    // selects keep the states in registers
    Rs.r = sb ? Ls.r : Rs.r; Rs.u = sb ? -Ls.u : Rs.u; Rs.v = sb ? Ls.v : Rs.v;
    Rs.w = sb ? Ls.w : Rs.w; Rs.p = sb ? Ls.p : Rs.p;
    Ls.r = sa ? Rs.r : Ls.r; Ls.u = sa ? -Rs.u : Ls.u; Ls.v = sa ? Rs.v : Ls.v;
    Ls.w = sa ? Rs.w : Ls.w; Ls.p = sa ? Rs.p : Ls.p;
    bool cnt;
    St<T> f = Solver<T>::solve(Ls, Rs, r0f, p0f, gam, cnt);
    T rf = r0f + f.r;
    T Fr = rf * f.u;
    F[0] = Fr;
    F[1] = Fr * f.u + f.p;
    F[2] = Fr * f.v;
    F[3] = Fr * f.w;
    F[4] = f.u * (gfac * (p0f + f.p) + T(0.5) * rf * ((f.u * f.u + f.v * f.v) + f.w * f.w));
    sg = f.u * nu;
    return cnt;
}

// Conservative update of one fluid cell: flux differences, gravity on the
// perturbation density (time centred) and on the mass flux in the energy.
template <typename T>
__device__ __forceinline__ void hydro_update(const T *cu, const T *Fl, const T *Fr, T nu, T dt, T gj, T *o)
{
    T rn = cu[0] - nu * (Fr[0] - Fl[0]);
    o[0] = rn;
    o[1] = cu[1] - nu * (Fr[1] - Fl[1]) + dt * gj * (T(0.5) * (cu[0] + rn));
    o[2] = cu[2] - nu * (Fr[2] - Fl[2]);
    o[3] = cu[3] - nu * (Fr[3] - Fl[3]);
    o[4] = cu[4] - nu * (Fr[4] - Fl[4]) + dt * gj * (T(0.5) * (Fl[0] + Fr[0]));
}

}  // namespace ppmb
