/*
 * ppmb_oracle.c -- plain FP64 CPU reference ("oracle") for one directionally
 * split 3-D PPM gas-dynamics step coupled to PPB multifluid advection, after
 * Woodward, Lin, Mao, Andrassy & Herwig, "Simulating 3-D Stellar
 * Hydrodynamics using PPM and PPB Multifluid Gas Dynamics on CPU and CPU+GPU
 * Nodes" (arXiv 1810.13416).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the HIP path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares
 * no code, header, table or constant generator with the HIP library.
 *
 * The paper names the method but defers its formulas to its references
 * ("we will not repeat the details", Sec. 4).  Every formula below is either
 * one the paper states in words (Sec. 1, Sec. 3, Sec. 4) or a reading taken
 * from the canonical PPM paper (Colella & Woodward 1984, "CW84"), marked
 * [reading].  Each reading is listed in the design notes of the repository.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (IEEE, no fast-math).
 * Parallelism is over independent pencils only, so results are bitwise
 * independent of the thread count.
 *
 * Parity: pinned.  The pins are tests that do not call this file's formulas
 * again: uniform-state and hydrostatic-state preservation, round-off
 * conservation, the exact Sod solution, closed-form two-shock collisions,
 * exactness on cubics and quadratics, mirror symmetry, bounds of fv, measured
 * convergence order and closed-form hydrostatic polytropes.  The optional
 * shock dissipation is pinned in its divergence (exact on linear fields and
 * at walls) and its effects (idle on uniform states and in rarefactions,
 * conservative, symmetric, smoothing behind a shock that stays in place);
 * its flux is pinned by a closed form: under uniform compression the
 * coefficient is the same at every interior face and the dissipation is a
 * discrete diffusion of each conserved hydro field, which fixes the
 * weight, its sign, the undivided divergence and the face differencing
 * field by field.  The optional flattening near strong shocks is pinned in its
 * coefficient (zero on smooth and expanding profiles and on weak jumps, one
 * at a compressive pressure step, mirror symmetric) and its effects (idle
 * where the coefficient is zero, conservative, symmetric, the Sod shock in
 * place with less post-shock noise).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Parameters and state                                                */
/* ------------------------------------------------------------------ */

enum { NG = 4 };           /* ghost cells per side: the stencil reaches 4 cells (Sec. 4) */
enum { NF = 15 };          /* evolving fields per cell */

/* conserved perturbation fields (the base state is subtracted, Sec. 1) */
enum { RHO = 0, MX = 1, MY = 2, MZ = 3, EN = 4,
       /* fv cell average and its 9 lowest moments (Sec. 4), stored as
          coefficients of the orthogonal basis 1, x, y, z, P2(x), P2(y),
          P2(z), xy, yz, zx on the unit cell, P2(s) = s^2 - 1/12 */
       F0 = 5, FX = 6, FY = 7, FZ = 8, FXX = 9, FYY = 10, FZZ = 11,
       FXY = 12, FYZ = 13, FZX = 14 };

typedef struct {
    int    n[3];          /* cells along x, y, z */
    double dx;            /* uniform cell width (Sec. 1: uniform Cartesian grid) */
    double origin[3];     /* low corner of the grid */
    int    bc[3];         /* per axis, both ends: 0 periodic, 1 reflecting */
    double gamma;
    int    sphere;        /* 1: cells whose centre has r >= sphere_r are solid (Sec. 3) */
    double sphere_r;
    int    grav_kind;     /* 0 none, 1 constant vector, 2 radial */
    double grav[4];       /* kind 1: gx, gy, gz.  kind 2: g0, rc, r1, r2 */
    int    base_kind;     /* 0 none (plain), 1 constant, 2 polytrope in z, 3 polytrope in r */
    double base[6];       /* kind 1: rho, p.  kinds 2,3: rho_b, p_b, s_b, s_i, f_jump, s_end */
    int    heat_kind;     /* 0 none, 1 layer in z, 2 ball in r */
    double heat[3];       /* Q0, extent, z0 (kind 1) */
    int    smooth_detect; /* 1: 5-cell smoothness test gates the constraints (the method);
                             0: always constrain; 2: never constrain (ablations) */
} or_params;

typedef struct {
    or_params P;
    long      ncell;
    double   *U[NF];      /* current state */
    double   *W[NF];      /* ping-pong buffer */
    double   *rho0, *p0;  /* base state cell values (FP64) */
    long      nstep;
    unsigned long long cnt[4]; /* fv limiter hits, unsmooth cell-variables, non-converged Riemann, steps */
    int       nthreads;
    double    spin_omega;  /* spin-up: final angular velocity about the z axis */
    long      spin_nramp;  /* ... reached over the steps 0 .. spin_nramp-1 */
    double    diss_k;      /* shock dissipation coefficient (0: off) */
    double   *divu;        /* undivided velocity divergence at the step start */
    int       flat_on;     /* flattening near strong shocks (CW84 Sec. 4) */
    double   *flat;        /* its coefficient for the pass in progress */
    double    rot_omega;   /* rotating frame: angular velocity about z (0: inertial) */
    int       rot_centrifugal; /* ... with the centrifugal term */
} or_sim;

static long cidx(const or_sim *S, int i, int j, int k)
{
    return ((long)k * S->P.n[1] + j) * S->P.n[0] + i;
}

static double cell_centre(const or_params *P, int axis, int i)
{
    return P->origin[axis] + ((double)i + 0.5) * P->dx;
}

/* ------------------------------------------------------------------ */
/* Gravity, heating, confining sphere (Sec. 2, Sec. 3)                  */
/* ------------------------------------------------------------------ */

/* Radial taper: gravity falls to zero a few cells before the confining
   sphere (Sec. 3).  [reading] linear from r1 to r2. */
static double grav_taper(const or_params *P, double r)
{
    double r1 = P->grav[2], r2 = P->grav[3];
    if (r <= r1) return 1.0;
    if (r >= r2) return 0.0;
    return (r2 - r) / (r2 - r1);
}

/* radial profile g_r(r) (signed, negative = inward) */
static double grav_radial(const or_params *P, double r)
{
    double g0 = P->grav[0], rc = P->grav[1];
    double shape = (r < rc) ? r / rc : (rc * rc) / (r * r);
    return -g0 * shape * grav_taper(P, r);
}

/* gravity vector at a point */
static void gravity_at(const or_params *P, const double x[3], double g[3])
{
    g[0] = g[1] = g[2] = 0.0;
    if (P->grav_kind == 1) {
        g[0] = P->grav[0]; g[1] = P->grav[1]; g[2] = P->grav[2];
    } else if (P->grav_kind == 2) {
        double g0 = P->grav[0], rc = P->grav[1];
        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        /* g = -g0 * xhat * shape(r) * taper(r), written without 1/r at r = 0 */
        double h = (r < rc) ? 1.0 / rc : (rc * rc) / (r * r * r);
        double t = grav_taper(P, r);
        for (int d = 0; d < 3; ++d) g[d] = -g0 * x[d] * h * t;
    }
}

/* [reading] heating profile: Q0 inside half the extent, smoothstep to 0 at the extent */
static double heat_shape(double xi)
{
    if (xi <= 0.5) return 1.0;
    if (xi >= 1.0) return 0.0;
    double t = 2.0 * xi - 1.0;
    return 1.0 - t * t * (3.0 - 2.0 * t);
}

static double heating_at(const or_params *P, const double x[3])
{
    if (P->heat_kind == 1) return P->heat[0] * heat_shape((x[2] - P->heat[2]) / P->heat[1]);
    if (P->heat_kind == 2) {
        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        return P->heat[0] * heat_shape(r / P->heat[1]);
    }
    return 0.0;
}

static int solid_at(const or_params *P, const double x[3])
{
    if (!P->sphere) return 0;
    double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    return r >= P->sphere_r;
}

static void cell_pos(const or_params *P, int i, int j, int k, double x[3])
{
    x[0] = cell_centre(P, 0, i); x[1] = cell_centre(P, 1, j); x[2] = cell_centre(P, 2, k);
}

/* ------------------------------------------------------------------ */
/* Base state: hydrostatic piecewise polytrope integrated in FP64 (Sec. 1:  */
/* the initial spherically symmetric state is saved on the grid and        */
/* subtracted out).  dp/ds = rho(p, s) g_s(s), rho = (p/K)^(1/gamma), K     */
/* jumps at s_i so that rho jumps by f at continuous p.  RK4, 8 steps per   */
/* cell width between breakpoints, then one RK4 step from the nearest node */
/* below each cell centre.                                                   */
/* ------------------------------------------------------------------ */

enum { MAXSEG = 6 };
typedef struct {
    double s0[MAXSEG], h[MAXSEG], K[MAXSEG], s1[MAXSEG];
    int    m[MAXSEG], nseg;
    double *p[MAXSEG];      /* node pressures, m+1 per segment */
} base_table;

static double base_g(const or_params *P, double s)
{
    if (P->base_kind == 2) return (P->grav_kind == 1) ? P->grav[2] : 0.0;
    return (P->grav_kind == 2) ? grav_radial(P, s) : 0.0;
}

static double base_rhs(const or_params *P, double K, double s, double p)
{
    double rho = pow(p / K, 1.0 / P->gamma);
    return rho * base_g(P, s);
}

static double rk4_step(const or_params *P, double K, double s, double p, double h)
{
    double k1 = base_rhs(P, K, s, p);
    double k2 = base_rhs(P, K, s + 0.5 * h, p + 0.5 * h * k1);
    double k3 = base_rhs(P, K, s + 0.5 * h, p + 0.5 * h * k2);
    double k4 = base_rhs(P, K, s + h, p + h * k3);
    return p + h * (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0;
}

/* Segments run between consecutive breakpoints: the base point, the entropy
   jump s_i, every kink of the radial gravity (rc, r1, r2) and s_end, so that
   no RK4 step straddles a kink of the right-hand side. */
static void base_build(const or_params *P, base_table *T)
{
    double rho_b = P->base[0], p_b = P->base[1], s_b = P->base[2];
    double s_i = P->base[3], f = P->base[4], s_end = P->base[5];
    double K1 = p_b / pow(rho_b, P->gamma);
    double K2 = K1 * pow(f, -P->gamma);
    double hmax = P->dx / 8.0;
    double bp[MAXSEG + 1];
    int nb = 0;
    bp[nb++] = s_b;
    double cand[4] = { s_i, 0.0, 0.0, 0.0 };
    int nc = 1;
    if (P->base_kind == 3 && P->grav_kind == 2) { cand[1] = P->grav[1]; cand[2] = P->grav[2]; cand[3] = P->grav[3]; nc = 4; }
    for (int q = 0; q < nc; ++q)           /* insert in increasing order, inside (s_b, s_end) */
        if (cand[q] > s_b && cand[q] < s_end) {
            int at = nb;
            while (at > 1 && bp[at - 1] > cand[q]) { bp[at] = bp[at - 1]; --at; }
            if (bp[at - 1] == cand[q]) { for (int r = at; r < nb; ++r) bp[r] = bp[r + 1]; continue; }
            bp[at] = cand[q]; ++nb;
        }
    bp[nb++] = s_end;
    T->nseg = nb - 1;
    double p_start = p_b;
    for (int sg = 0; sg < T->nseg; ++sg) {
        double a = bp[sg], b = bp[sg + 1];
        int m = (int)ceil((b - a) / hmax);
        if (m < 1) m = 1;
        T->m[sg] = m;
        T->s0[sg] = a;
        T->s1[sg] = b;
        T->h[sg] = (b - a) / m;
        T->K[sg] = (a >= s_i) ? K2 : K1;
        T->p[sg] = (double *)malloc(sizeof(double) * (m + 1));
        T->p[sg][0] = p_start;
        for (int q = 0; q < m; ++q)
            T->p[sg][q + 1] = rk4_step(P, T->K[sg], a + q * T->h[sg], T->p[sg][q], T->h[sg]);
        p_start = T->p[sg][m];
    }
}

static void base_eval(const or_params *P, const base_table *T, double s, double *rho, double *p)
{
    (void)P;
    int sg = 0;
    while (sg < T->nseg - 1 && s >= T->s1[sg]) ++sg;
    int q = (int)floor((s - T->s0[sg]) / T->h[sg]);
    if (q < 0) q = 0;
    if (q > T->m[sg] - 1) q = T->m[sg] - 1;
    double sq = T->s0[sg] + q * T->h[sg];
    double pv = rk4_step(P, T->K[sg], sq, T->p[sg][q], s - sq);
    *p = pv;
    *rho = pow(pv / T->K[sg], 1.0 / P->gamma);
}

static void base_free(base_table *T)
{
    for (int sg = 0; sg < T->nseg; ++sg) free(T->p[sg]);
}

static void base_fill(or_sim *S)
{
    const or_params *P = &S->P;
    if (P->base_kind == 0 || P->base_kind == 1) {
        double r = (P->base_kind == 1) ? P->base[0] : 0.0;
        double p = (P->base_kind == 1) ? P->base[1] : 0.0;
        for (long c = 0; c < S->ncell; ++c) { S->rho0[c] = r; S->p0[c] = p; }
        return;
    }
    base_table T;
    base_build(P, &T);
    #pragma omp parallel for schedule(static) num_threads(S->nthreads)
    for (int k = 0; k < P->n[2]; ++k)
        for (int j = 0; j < P->n[1]; ++j)
            for (int i = 0; i < P->n[0]; ++i) {
                double x[3];
                cell_pos(P, i, j, k, x);
                double s = (P->base_kind == 2) ? x[2]
                         : sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                long c = cidx(S, i, j, k);
                base_eval(P, &T, s, &S->rho0[c], &S->p0[c]);
            }
    base_free(&T);
}

/* ------------------------------------------------------------------ */
/* One-dimensional building blocks                                     */
/* ------------------------------------------------------------------ */

/* Sec. 1: interface values one order higher than the parabola.  [reading]
   4th-order value from the 4 surrounding cell averages (CW84 eq. 1.6 on a
   uniform grid).  a, b straddle the face; am is left of a, bp right of b. */
double or_face4(double am, double a, double b, double bp)
{
    return (7.0 * (a + b) - (am + bp)) / 12.0;
}

/* Sec. 1: smoothness judged on the 5 cells centred on the cell of interest.
   [reading] With the three second differences D in the window: the data is
   smooth (weight 1, no constraints) when all D are zero, or all share one
   strict sign with max|D| <= 2 min|D|; not smooth (weight 0, constraints
   applied) when their signs differ or max|D| >= 3 min|D|; the weight falls
   linearly in between, so that the reconstruction depends continuously on
   the data.  Returns the weight of the unconstrained parabola. */
double or_smooth_weight(const double q[5])
{
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = (q[k] + q[k + 2]) - 2.0 * q[k + 1];
    if (d[0] == 0.0 && d[1] == 0.0 && d[2] == 0.0) return 1.0;
    int pos = d[0] > 0.0 && d[1] > 0.0 && d[2] > 0.0;
    int neg = d[0] < 0.0 && d[1] < 0.0 && d[2] < 0.0;
    if (!pos && !neg) return 0.0;
    double a0 = fabs(d[0]), a1 = fabs(d[1]), a2 = fabs(d[2]);
    double mx = fmax(a0, fmax(a1, a2)), mn = fmin(a0, fmin(a1, a2));
    if (mx <= 2.0 * mn) return 1.0;
    if (mx >= 3.0 * mn) return 0.0;
    return (3.0 * mn - mx) / mn;
}

/* van Leer limited slope (CW84 eq. 1.8) */
static double limited_slope(double qm, double q, double qp)
{
    double dl = q - qm, dr = qp - q;
    if (!(dl * dr > 0.0)) return 0.0;
    double dc = 0.5 * (qp - qm);
    double m = fmin(fabs(dc), fmin(2.0 * fabs(dl), 2.0 * fabs(dr)));
    return dc > 0.0 ? m : -m;
}

/* Interface value built from limited slopes (CW84 eq. 1.6 with eq. 1.8),
   written symmetrically in the two cells that share the face. */
static double face_limited(double qa, double qb, double sa, double sb)
{
    return 0.5 * (qa + qb) - (sb - sa) / 6.0;
}

/* Parabola constraints of CW84 eq. 1.10, applied only to cells judged not
   smooth.  In/out: left and right edge values. */
static void constrain_parabola(double q, double *qL, double *qR)
{
    if ((*qR - q) * (q - *qL) <= 0.0) { *qL = q; *qR = q; return; }
    double dq = *qR - *qL;
    double q6 = 6.0 * (q - 0.5 * (*qL + *qR));
    if (dq * q6 > dq * dq) *qL = 3.0 * q - 2.0 * *qR;
    else if (dq * q6 < -(dq * dq)) *qR = 3.0 * q - 2.0 * *qL;
}

/* Averages of the parabola over the last (right edge) or first (left edge)
   fraction y of the cell (CW84 eqs. 1.12). */
static double avg_right(double qR, double dq, double q6, double y)
{
    return qR - (0.5 * y) * (dq - (1.0 - (2.0 / 3.0) * y) * q6);
}
static double avg_left(double qL, double dq, double q6, double y)
{
    return qL + (0.5 * y) * (dq + (1.0 - (2.0 / 3.0) * y) * q6);
}

/* ------------------------------------------------------------------ */
/* Two-shock Riemann solver on the pressure perturbation (CW84 Sec. 2)   */
/* ------------------------------------------------------------------ */

/* States are (rho', u, v, w, p').  The base values at the face, rho0f and
   p0f, are shared by both sides, so p0f cancels from every pressure
   difference (Sec. 1: large base contributions cancelled explicitly).
   Output: the face state (rho', u, v, w, p') sampled at the face.
   Returns the number of Newton iterations; negative if not converged. */
int or_riemann(const double *L, const double *R, double rho0f, double p0f, double gamma,
               double *out)
{
    const double A = (gamma + 1.0) / (2.0 * gamma);
    double rL = rho0f + L[0], rR = rho0f + R[0];
    double pL = p0f + L[4], pR = p0f + R[4];
    double CL = sqrt(gamma * pL * rL), CR = sqrt(gamma * pR * rR);
    double cL = CL / rL, cR = CR / rR;
    double pfl = 1e-10 * fmin(pL, pR) - p0f;   /* floor on p* expressed as p' */
    /* acoustic guess */
    double ps = (CR * L[4] + CL * R[4] + CL * CR * (L[1] - R[1])) / (CL + CR);
    if (ps < pfl) ps = pfl;
    double WL = CL, WR = CR, us = 0.0;
    int it, conv = 0;
    for (it = 1; it <= 20; ++it) {
        WL = CL * sqrt(1.0 + A * (ps - L[4]) / pL);
        WR = CR * sqrt(1.0 + A * (ps - R[4]) / pR);
        double uLs = L[1] - (ps - L[4]) / WL;
        double uRs = R[1] + (ps - R[4]) / WR;
        double ZL = 2.0 * WL * WL * WL / (WL * WL + CL * CL);
        double ZR = 2.0 * WR * WR * WR / (WR * WR + CR * CR);
        double du = uRs - uLs;
        us = (ZL * uLs + ZR * uRs) / (ZL + ZR);
        ps = ps - ZL * ZR * du / (ZL + ZR);
        if (ps < pfl) ps = pfl;
        if (fabs(du) <= 1e-13 * (cL + cR)) { conv = 1; break; }
    }
    if (it > 20) it = 20;
    /* sample the side the contact leaves behind: us >= 0 -> left */
    if (us >= 0.0) {
        double S = L[1] - WL / rL;              /* left wave speed */
        if (S >= 0.0) { for (int v = 0; v < 5; ++v) out[v] = L[v]; }
        else {
            double X = rL * (ps - L[4]) / (WL * WL);
            out[0] = L[0] + rL * X / (1.0 - X);
            out[1] = us; out[2] = L[2]; out[3] = L[3]; out[4] = ps;
        }
    } else {
        double S = R[1] + WR / rR;              /* right wave speed */
        if (S <= 0.0) { for (int v = 0; v < 5; ++v) out[v] = R[v]; }
        else {
            double X = rR * (ps - R[4]) / (WR * WR);
            out[0] = R[0] + rR * X / (1.0 - X);
            out[1] = us; out[2] = R[2]; out[3] = R[3]; out[4] = ps;
        }
    }
    return conv ? it : -it;
}

/* ------------------------------------------------------------------ */
/* PPB transport of the fv moments along one pass (Sec. 1, Sec. 4)       */
/* ------------------------------------------------------------------ */

/* [reading] PPB as a Lagrange-remap in flux form.  During the pass each
   cell j moves as a Lagrangian slab; its faces move by sigma = u* dt/dx
   (in cell widths), so it has length L_j = 1 + sigma_{j+1/2} - sigma_{j-1/2}
   and centre offset delta_j = (sigma_{j-1/2} + sigma_{j+1/2})/2.  The
   volume fraction is carried with the material, so the cell's polynomial
   is stretched onto the new interval.  The slab of a donor cell that ends
   up past a face is integrated exactly; its moments about the face are
   G0 = sigma*I0, G1 = sigma^2*I1, H2 = sigma^3*I2, where I_k is the integral
   of the donor profile times u^k over the slab, u in [0,1] running from the
   face outwards.  New moments = Lagrangian moments about the cell centre
   minus outgoing plus incoming slabs, shifted by +-1/2. */

/* integrals I0, I1, I2 of a quadratic a0 + a1 s + a2 (s^2 - 1/12) over the
   last fraction t of the cell, s = 1/2 - t + t u */
static void slab_quad(double a0, double a1, double a2, double t, double I[3])
{
    double h = 0.5 - t;
    double al0 = a0 + a1 * h + a2 * (h * h - 1.0 / 12.0);
    double al1 = t * (a1 + 2.0 * a2 * h);
    double al2 = a2 * (t * t);
    I[0] = al0 + al1 / 2.0 + al2 / 3.0;
    I[1] = al0 / 2.0 + al1 / 3.0 + al2 / 4.0;
    I[2] = al0 / 3.0 + al1 / 4.0 + al2 / 5.0;
}

static void slab_lin(double b0, double b1, double t, double J[2])
{
    double be0 = b0 + b1 * (0.5 - t);
    double be1 = b1 * t;
    J[0] = be0 + be1 / 2.0;
    J[1] = be0 / 2.0 + be1 / 3.0;
}

/* Sec. 1: the fv representation is constrained almost never.  [reading] If the profile along the
   pass, g(s) = a0 + a1 s + a2 P2(s), leaves [0,1] on the cell, scale a1 and
   a2 by the largest theta in [0,1] that brings it back (Zhang & Shu 2010
   scaling).  Returns 1 if it changed the profile by more than round-off. */
static int fv_limit(double a0, double *a1, double *a2)
{
    double gm = a0 - 0.5 * *a1 + *a2 / 6.0;
    double gp = a0 + 0.5 * *a1 + *a2 / 6.0;
    double gmin = fmin(gm, gp), gmax = fmax(gm, gp);
    if (*a2 != 0.0) {
        double sv = -*a1 / (2.0 * *a2);
        if (sv > -0.5 && sv < 0.5) {
            double gv = a0 + *a1 * sv + *a2 * (sv * sv - 1.0 / 12.0);
            gmin = fmin(gmin, gv); gmax = fmax(gmax, gv);
        }
    }
    double th = 1.0;
    if (gmax > 1.0) th = fmin(th, (1.0 - a0) / (gmax - a0));
    if (gmin < 0.0) th = fmin(th, a0 / (a0 - gmin));
    if (th >= 1.0) return 0;
    if (th < 0.0) th = 0.0;
    double s1 = fabs(*a1) + fabs(*a2);
    *a1 *= th; *a2 *= th;
    /* counted when the profile changes by more than round-off: saturated
       regions (fv = 0 or 1) otherwise trip the bound at the last bit */
    return (1.0 - th) * s1 > 1e-9;
}

/* Per-pencil PPB work.  Coefficients in pass-local order:
   c[0..2]  quadratic along the pass: a0, a_s, a_ss
   c[3..4]  first transverse slope varying along the pass: b0, b1
   c[5..6]  second transverse slope: b0, b1
   c[7..9]  constants along the pass: the two transverse P2 and their mixed term
   Entries with index j+NG, j in [-NG, n+NG).  sig[j+NG] is sigma at face j+1/2.
   Updates cells 0..n-1 of `out` (same layout); donors -1..n are read.
   Odd-in-s coefficients are 2 (a_s), 4 and 6. */
static int ppb_pencil(int n, double *const c[10], const double *sig, const int *solid,
                      double *const out[10])
{
    int hits = 0;
    int m = n + 2 * NG;
    double *Lw = (double *)malloc(sizeof(double) * m);
    double *qa1 = (double *)malloc(sizeof(double) * m);
    double *qa2 = (double *)malloc(sizeof(double) * m);
    double (*G)[10] = malloc(sizeof(double[10]) * m);   /* G0,G1,H2 | G0,G1 | G0,G1 | G0 G0 G0 */
    /* Lagrangian lengths and limited quadratics of donors -1..n */
    for (int j = -1; j <= n; ++j) {
        int J = j + NG;
        Lw[J] = 1.0 + (sig[J] - sig[J - 1]);
        qa1[J] = c[1][J]; qa2[J] = c[2][J];
        int hit = fv_limit(c[0][J], &qa1[J], &qa2[J]);
        if (hit && j >= 0 && j < n && !solid[J]) hits++;
    }
    /* slabs through faces -1/2 .. n-1/2 */
    for (int f = -1; f <= n - 1; ++f) {
        int F = f + NG;
        double s = sig[F];
        for (int q = 0; q < 10; ++q) G[F][q] = 0.0;
        if (s == 0.0) continue;
        int D = (s > 0.0) ? F : F + 1;             /* donor cell index (array) */
        double o = (s > 0.0) ? 1.0 : -1.0;        /* flip odd-in-s terms for a right donor */
        double t = fabs(s) / Lw[D];
        double I[3], J1[2], J2[2];
        slab_quad(c[0][D], o * qa1[D], qa2[D], t, I);
        slab_lin(c[3][D], o * c[4][D], t, J1);
        slab_lin(c[5][D], o * c[6][D], t, J2);
        double s2 = s * s, s3 = s2 * s;
        G[F][0] = s * I[0]; G[F][1] = s2 * I[1]; G[F][2] = s3 * I[2];
        G[F][3] = s * J1[0]; G[F][4] = s2 * J1[1];
        G[F][5] = s * J2[0]; G[F][6] = s2 * J2[1];
        G[F][7] = s * c[7][D]; G[F][8] = s * c[8][D]; G[F][9] = s * c[9][D];
    }
    for (int j = 0; j < n; ++j) {
        int J = j + NG;
        if (solid[J]) { for (int q = 0; q < 10; ++q) out[q][J] = c[q][J]; continue; }
        double sl = sig[J - 1], sr = sig[J];
        double ds = sr - sl;
        double L = 1.0 + ds;
        double dl = 0.5 * (sl + sr);
        const double *GL = G[J - 1], *GR = G[J];
        double a0 = c[0][J], a1 = qa1[J], a2 = qa2[J];
        double M0 = L * a0;
        double M1 = L * (dl * a0 + L * a1 / 12.0);
        double M2 = L * (dl * dl * a0 + dl * L * a1 / 6.0 + L * L * a2 / 180.0
                         + a0 * ds * (2.0 + ds) / 12.0);
        out[0][J] = M0 - (GR[0] - GL[0]);
        out[1][J] = 12.0 * (M1 - (GR[1] - GL[1]) - 0.5 * (GR[0] + GL[0]));
        out[2][J] = 180.0 * (M2 - (GR[2] - GL[2]) - (GR[1] + GL[1]) - (GR[0] - GL[0]) / 6.0);
        for (int p = 0; p < 2; ++p) {
            int b = 3 + 2 * p;
            double b0 = c[b][J], b1 = c[b + 1][J];
            double N0 = L * b0;
            double N1 = L * (dl * b0 + L * b1 / 12.0);
            out[b][J] = N0 - (GR[b] - GL[b]);
            out[b + 1][J] = 12.0 * (N1 - (GR[b + 1] - GL[b + 1]) - 0.5 * (GR[b] + GL[b]));
        }
        for (int q = 7; q < 10; ++q) out[q][J] = L * c[q][J] - (GR[q] - GL[q]);
    }
    free(Lw); free(qa1); free(qa2); free(G);
    return hits;
}

/* Exported for unit pins: one PPB pencil with prescribed face Courant
   numbers.  Arrays have n + 2*NG entries (cells -NG..n+NG-1). */
int or_ppb_pencil(int n, double *const c[10], const double *sig, double *const out[10])
{
    int *solid = (int *)calloc(n + 2 * NG, sizeof(int));
    int h = ppb_pencil(n, c, sig, solid, out);
    free(solid);
    return h;
}

/* ------------------------------------------------------------------ */
/* 2-D PPB under a prescribed solid-body rotation (Fig. 3)              */
/* ------------------------------------------------------------------ */

/* [reading] The advection test of Fig. 3: a 2-D grid of nx x ny cells of
   width dx (cell (i, j) centred at x0 + (i + 1/2) dx, y0 + (j + 1/2) dx),
   fv carried as its 6 low-order moments (1, x, y, P2(x), P2(y), xy on the
   unit cell; the 3-D PPB with every z term zero), periodic boundaries, and
   the velocity of a rigid rotation with angular speed omega about (xc, yc):
   u = -omega (y - yc), v = omega (x - xc).  A step is an x pass then a y
   pass on even steps and the reverse on odd steps; a pass moves each pencil
   by the face Courant numbers of that velocity (u at x-faces depends on y
   only, so every cell of a pencil keeps its length).
   c[0..5] = f0, fx, fy, fxx, fyy, fxy, each nx*ny values, x fastest. */
static void ppb2d_pass(int nx, int ny, double dx, double x0, double y0, double xc, double yc,
                       double omega, double dt, int axis, double *const c[6])
{
    const int n = axis == 0 ? nx : ny;            /* cells along the pass */
    const int np = axis == 0 ? ny : nx;           /* pencils */
    const int m = n + 2 * NG;
    /* pass-local order (quadratic along, transverse linear, transverse
       linear in z = 0, constants): x pass f0 fx fxx | fy fxy | 0 0 | fyy 0 0,
       y pass f0 fy fyy | fx fxy | 0 0 | fxx 0 0 */
    const int map_x[10] = { 0, 1, 3, 2, 5, -1, -1, 4, -1, -1 };
    const int map_y[10] = { 0, 2, 4, 1, 5, -1, -1, 3, -1, -1 };
    const int *map = axis == 0 ? map_x : map_y;
#pragma omp parallel for schedule(static)
    for (int p = 0; p < np; ++p) {
        double *in[10], *out[10];
        double *buf = (double *)calloc((size_t)21 * m, sizeof(double));
        for (int q = 0; q < 10; ++q) { in[q] = buf + q * m; out[q] = buf + (10 + q) * m; }
        double *sig = buf + 20 * m;
        /* the pencil's transverse coordinate and its face Courant number */
        const double tc = (axis == 0 ? y0 : x0) + (p + 0.5) * dx;
        const double vel = axis == 0 ? -omega * (tc - yc) : omega * (tc - xc);
        const double s = vel * dt / dx;
        for (int J = 0; J < m; ++J) {
            int j = ((J - NG) % n + n) % n;        /* periodic */
            long cell = axis == 0 ? (long)p * nx + j : (long)j * nx + p;
            for (int q = 0; q < 10; ++q) in[q][J] = map[q] < 0 ? 0.0 : c[map[q]][cell];
            sig[J] = s;
        }
        int *solid = (int *)calloc(m, sizeof(int));
        ppb_pencil(n, in, sig, solid, out);
        free(solid);
        for (int j = 0; j < n; ++j) {
            long cell = axis == 0 ? (long)p * nx + j : (long)j * nx + p;
            for (int q = 0; q < 10; ++q)
                if (map[q] >= 0) c[map[q]][cell] = out[q][j + NG];
        }
        free(buf);
    }
}

/* nsteps steps from step number step0 (its parity picks the pass order). */
void or_ppb2d_steps(int nx, int ny, double dx, double x0, double y0, double xc, double yc,
                    double omega, double dt, int nsteps, long step0, double *const c[6])
{
    for (int k = 0; k < nsteps; ++k) {
        int first = ((step0 + k) & 1) ? 1 : 0;
        ppb2d_pass(nx, ny, dx, x0, y0, xc, yc, omega, dt, first, c);
        ppb2d_pass(nx, ny, dx, x0, y0, xc, yc, omega, dt, 1 - first, c);
    }
}

/* ------------------------------------------------------------------ */
/* One pencil of one pass: PPM hydro + PPB                             */
/* ------------------------------------------------------------------ */

typedef struct {
    int n;
    double *rhop, *mn, *mt1, *mt2, *ep, *r0, *p0, *g;   /* gathered, n+2NG */
    double *div;                                        /* divergence (shock dissipation) */
    double diss_k;
    double *flat;                                       /* flattening coefficient */
    int flat_on;
    int *solid;
    double *f[10];                                      /* pass-local PPB order */
    /* outputs */
    double *o_rhop, *o_mn, *o_mt1, *o_mt2, *o_ep;
    double *o_f[10];
    /* work */
    double *w[40];
    double (*TL)[5], (*TR)[5], (*FL)[6];
    unsigned long long unsmooth, nonconv, hits;
} pencil;

static void pencil_alloc(pencil *pc, int n)
{
    int m = n + 2 * NG;
    pc->n = n;
    double **arr[] = { &pc->rhop, &pc->mn, &pc->mt1, &pc->mt2, &pc->ep, &pc->r0, &pc->p0, &pc->g,
                       &pc->o_rhop, &pc->o_mn, &pc->o_mt1, &pc->o_mt2, &pc->o_ep, &pc->div, &pc->flat };
    for (unsigned a = 0; a < sizeof(arr) / sizeof(arr[0]); ++a)
        *arr[a] = (double *)calloc(m, sizeof(double));
    for (int q = 0; q < 10; ++q) {
        pc->f[q] = (double *)calloc(m, sizeof(double));
        pc->o_f[q] = (double *)calloc(m, sizeof(double));
    }
    for (int q = 0; q < 40; ++q) pc->w[q] = (double *)calloc(m, sizeof(double));
    pc->solid = (int *)calloc(m, sizeof(int));
    pc->TL = malloc(sizeof(double[5]) * m);
    pc->TR = malloc(sizeof(double[5]) * m);
    pc->FL = malloc(sizeof(double[6]) * m);
}

static void pencil_free(pencil *pc)
{
    double *arr[] = { pc->rhop, pc->mn, pc->mt1, pc->mt2, pc->ep, pc->r0, pc->p0, pc->g,
                      pc->o_rhop, pc->o_mn, pc->o_mt1, pc->o_mt2, pc->o_ep, pc->div, pc->flat };
    for (unsigned a = 0; a < sizeof(arr) / sizeof(arr[0]); ++a) free(arr[a]);
    for (int q = 0; q < 10; ++q) { free(pc->f[q]); free(pc->o_f[q]); }
    for (int q = 0; q < 40; ++q) free(pc->w[q]);
    free(pc->solid); free(pc->TL); free(pc->TR); free(pc->FL);
}

/* The 1-D pass over one pencil (Sec. 4: all steps of a 1-D pass composed
   into one loop over the pencil).  Index J = j + NG. */
static void pencil_update(pencil *pc, double dt, double dx, double gamma, int detect)
{
    const int n = pc->n, m = n + 2 * NG;
    const double nu = dt / dx, gm1 = gamma - 1.0;
    double *rho = pc->w[0], *u = pc->w[1], *v = pc->w[2], *w = pc->w[3], *pp = pc->w[4];
    double *c = pc->w[5], *r0f = pc->w[6], *p0f = pc->w[7];
    double *Q[5] = { pc->rhop, u, v, w, pp };          /* interpolated variables */
    double *qf[5] = { pc->w[8], pc->w[9], pc->w[10], pc->w[11], pc->w[12] };
    double *sm[5] = { pc->w[13], pc->w[14], pc->w[15], pc->w[16], pc->w[17] };
    double *qL[5] = { pc->w[18], pc->w[19], pc->w[20], pc->w[21], pc->w[22] };
    double *qR[5] = { pc->w[23], pc->w[24], pc->w[25], pc->w[26], pc->w[27] };
    double *sig = pc->w[28];

    /* (1) primitives with the base added back, Sec. 1 */
    for (int J = 0; J < m; ++J) {
        rho[J] = pc->r0[J] + pc->rhop[J];
        u[J] = pc->mn[J] / rho[J];
        v[J] = pc->mt1[J] / rho[J];
        w[J] = pc->mt2[J] / rho[J];
        pp[J] = gm1 * (pc->ep[J] - 0.5 * (pc->mn[J] * u[J] + pc->mt1[J] * v[J] + pc->mt2[J] * w[J]));
        double p = pc->p0[J] + pp[J];
        c[J] = sqrt(gamma * p / rho[J]);
    }
    /* (2) base face values and 4th-order interface values, faces -3..n+1 */
    for (int J = 1; J <= m - 3; ++J) {
        r0f[J] = or_face4(pc->r0[J - 1], pc->r0[J], pc->r0[J + 1], pc->r0[J + 2]);
        p0f[J] = or_face4(pc->p0[J - 1], pc->p0[J], pc->p0[J + 1], pc->p0[J + 2]);
        for (int q = 0; q < 5; ++q)
            qf[q][J] = or_face4(Q[q][J - 1], Q[q][J], Q[q][J + 1], Q[q][J + 2]);
    }
    /* (3) limited slopes, cells -3..n+2 */
    for (int J = 1; J <= m - 2; ++J)
        for (int q = 0; q < 5; ++q)
            sm[q][J] = limited_slope(Q[q][J - 1], Q[q][J], Q[q][J + 1]);
    /* (4) parabolas, cells -2..n+1; constraints only where the 5-cell
       window is not smooth (Sec. 1), blended in over the graded band */
    for (int J = 2; J <= m - 3; ++J) {
        for (int q = 0; q < 5; ++q) {
            double win[5] = { Q[q][J - 2], Q[q][J - 1], Q[q][J], Q[q][J + 1], Q[q][J + 2] };
            double ws = detect == 1 ? or_smooth_weight(win) : (detect == 2 ? 1.0 : 0.0);
            double l = qf[q][J - 1], r = qf[q][J];
            if (ws < 1.0) {
                double lc = face_limited(Q[q][J - 1], Q[q][J], sm[q][J - 1], sm[q][J]);
                double rc = face_limited(Q[q][J], Q[q][J + 1], sm[q][J], sm[q][J + 1]);
                constrain_parabola(Q[q][J], &lc, &rc);
                if (ws > 0.0) { lc = lc + ws * (l - lc); rc = rc + ws * (r - rc); }
                l = lc; r = rc;
                /* counted in the fluid cells of the pencil (a solid cell
                   is not part of the flow, Sec. 3, and keeps its state) */
                if (J >= NG && J < NG + n && !pc->solid[J]) pc->unsmooth++;
            }
            if (pc->flat_on) {
                /* flattening (CW84 Sec. 4) of the final edge values toward
                   the cell average */
                const double f = pc->flat[J];
                l = f * Q[q][J] + (1.0 - f) * l;
                r = f * Q[q][J] + (1.0 - f) * r;
            }
            qL[q][J] = l; qR[q][J] = r;
        }
    }
    /* (5) characteristic tracing (CW84 Sec. 3) plus half-step sources.
       TL[J]: state at the right face of cell J; TR[J]: at its left face. */
    for (int J = 2; J <= m - 3; ++J) {
        double rj = rho[J], cj = c[J], uj = u[J], c2 = cj * cj;
        double lam[3] = { uj - cj, uj, uj + cj };
        double dq[5], q6[5];
        for (int q = 0; q < 5; ++q) {
            dq[q] = qR[q][J] - qL[q][J];
            q6[q] = 6.0 * (Q[q][J] - 0.5 * (qL[q][J] + qR[q][J]));
        }
        /* right face: waves with positive speed */
        {
            double y = fmax(lam[2], 0.0) * nu;
            double ref[5];
            for (int q = 0; q < 5; ++q) ref[q] = avg_right(qR[q][J], dq[q], q6[q], y);
            double b0 = 0.0, bm = 0.0;
            if (lam[1] > 0.0) {
                double y0 = lam[1] * nu;
                double dr = ref[0] - avg_right(qR[0][J], dq[0], q6[0], y0);
                double dp = ref[4] - avg_right(qR[4][J], dq[4], q6[4], y0);
                b0 = dr - dp / c2;
            }
            if (lam[0] > 0.0) {
                double ym = lam[0] * nu;
                double du = ref[1] - avg_right(qR[1][J], dq[1], q6[1], ym);
                double dp = ref[4] - avg_right(qR[4][J], dq[4], q6[4], ym);
                bm = dp / (2.0 * c2) - (rj / (2.0 * cj)) * du;
            }
            double yv = fmax(lam[1], 0.0) * nu;
            pc->TL[J][0] = ref[0] - b0 - bm;
            pc->TL[J][1] = ref[1] + bm * (cj / rj);
            pc->TL[J][2] = avg_right(qR[2][J], dq[2], q6[2], yv);
            pc->TL[J][3] = avg_right(qR[3][J], dq[3], q6[3], yv);
            pc->TL[J][4] = ref[4] - bm * c2;
        }
        /* left face: waves with negative speed */
        {
            double y = fmax(-lam[0], 0.0) * nu;
            double ref[5];
            for (int q = 0; q < 5; ++q) ref[q] = avg_left(qL[q][J], dq[q], q6[q], y);
            double b0 = 0.0, bp = 0.0;
            if (lam[1] < 0.0) {
                double y0 = -lam[1] * nu;
                double dr = ref[0] - avg_left(qL[0][J], dq[0], q6[0], y0);
                double dp = ref[4] - avg_left(qL[4][J], dq[4], q6[4], y0);
                b0 = dr - dp / c2;
            }
            if (lam[2] < 0.0) {
                double yp = -lam[2] * nu;
                double du = ref[1] - avg_left(qL[1][J], dq[1], q6[1], yp);
                double dp = ref[4] - avg_left(qL[4][J], dq[4], q6[4], yp);
                bp = dp / (2.0 * c2) + (rj / (2.0 * cj)) * du;
            }
            double yv = fmax(-lam[1], 0.0) * nu;
            pc->TR[J][0] = ref[0] - b0 - bp;
            pc->TR[J][1] = ref[1] - bp * (cj / rj);
            pc->TR[J][2] = avg_left(qL[2][J], dq[2], q6[2], yv);
            pc->TR[J][3] = avg_left(qL[3][J], dq[3], q6[3], yv);
            pc->TR[J][4] = ref[4] - bp * c2;
        }
        /* half-step sources: gravity on rho' (momentum), base advection */
        double hdt = 0.5 * dt;
        double su = hdt * (pc->rhop[J] * pc->g[J] / rj);
        double sr = hdt * (uj * (r0f[J] - r0f[J - 1]) / dx);
        double sp = hdt * (uj * (p0f[J] - p0f[J - 1]) / dx);
        pc->TL[J][1] += su; pc->TR[J][1] += su;
        pc->TL[J][0] -= sr; pc->TR[J][0] -= sr;
        pc->TL[J][4] -= sp; pc->TR[J][4] -= sp;
    }
    /* (6) Riemann problems and fluxes at faces -2..n (face J is J+1/2) */
    for (int J = 2; J <= m - 4; ++J) {
        double Ls[5], Rs[5], f[5];
        for (int q = 0; q < 5; ++q) { Ls[q] = pc->TL[J][q]; Rs[q] = pc->TR[J + 1][q]; }
        int sa = pc->solid[J], sb = pc->solid[J + 1];
        if (sa && sb) { for (int q = 0; q < 6; ++q) pc->FL[J][q] = 0.0; sig[J] = 0.0; continue; }
        /* a face between a fluid and a solid cell is a reflecting wall (Sec. 3) */
        if (sb) { for (int q = 0; q < 5; ++q) Rs[q] = Ls[q]; Rs[1] = -Ls[1]; }
        if (sa) { for (int q = 0; q < 5; ++q) Ls[q] = Rs[q]; Ls[1] = -Rs[1]; }
        int it = or_riemann(Ls, Rs, r0f[J], p0f[J], gamma, f);
        if (it < 0 && J >= NG - 1 && J < NG + n) pc->nonconv++;
        double rf = r0f[J] + f[0];
        double Fr = rf * f[1];
        pc->FL[J][0] = Fr;
        pc->FL[J][1] = Fr * f[1] + f[4];
        pc->FL[J][2] = Fr * f[2];
        pc->FL[J][3] = Fr * f[3];
        pc->FL[J][4] = f[1] * (gamma / gm1 * (p0f[J] + f[4])
                               + 0.5 * rf * ((f[1] * f[1] + f[2] * f[2]) + f[3] * f[3]));
        sig[J] = f[1] * nu;
        /* shock dissipation [reading, after CW84 Sec. 4 with the full 3-D
           divergence, Sec. 1]: where the flow converges, a diffusive flux
           of the conserved hydro perturbations across the face */
        if (pc->diss_k > 0.0 && !sa && !sb) {
            double nv = pc->diss_k * fmax(0.0, -0.5 * (pc->div[J] + pc->div[J + 1]));
            pc->FL[J][0] += nv * (pc->rhop[J] - pc->rhop[J + 1]);
            pc->FL[J][1] += nv * (pc->mn[J] - pc->mn[J + 1]);
            pc->FL[J][2] += nv * (pc->mt1[J] - pc->mt1[J + 1]);
            pc->FL[J][3] += nv * (pc->mt2[J] - pc->mt2[J + 1]);
            pc->FL[J][4] += nv * (pc->ep[J] - pc->ep[J + 1]);
        }
    }
    /* (7) conservative update of cells 0..n-1, gravity on the perturbation */
    for (int J = NG; J < NG + n; ++J) {
        if (pc->solid[J]) {
            pc->o_rhop[J] = pc->rhop[J]; pc->o_mn[J] = pc->mn[J]; pc->o_mt1[J] = pc->mt1[J];
            pc->o_mt2[J] = pc->mt2[J]; pc->o_ep[J] = pc->ep[J];
            continue;
        }
        const double *Fl = pc->FL[J - 1], *Fr = pc->FL[J];
        double rn = pc->rhop[J] - nu * (Fr[0] - Fl[0]);
        pc->o_rhop[J] = rn;
        pc->o_mn[J] = pc->mn[J] - nu * (Fr[1] - Fl[1]) + dt * pc->g[J] * (0.5 * (pc->rhop[J] + rn));
        pc->o_mt1[J] = pc->mt1[J] - nu * (Fr[2] - Fl[2]);
        pc->o_mt2[J] = pc->mt2[J] - nu * (Fr[3] - Fl[3]);
        pc->o_ep[J] = pc->ep[J] - nu * (Fr[4] - Fl[4]) + dt * pc->g[J] * (0.5 * (Fl[0] + Fr[0]));
    }
    /* (8) PPB moments */
    pc->hits += ppb_pencil(n, pc->f, sig, pc->solid, pc->o_f);
}

/* ------------------------------------------------------------------ */
/* Pass driver                                                          */
/* ------------------------------------------------------------------ */

static int mixed_of(int a, int b) { return FXY + (4 - a - b) % 3; }

/* pass-local PPB field order and which entries are odd in the pass axis */
static void ppb_order(int d, int idx[10])
{
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    idx[0] = F0; idx[1] = FX + d; idx[2] = FXX + d;
    idx[3] = FX + t1; idx[4] = mixed_of(d, t1);
    idx[5] = FX + t2; idx[6] = mixed_of(d, t2);
    idx[7] = FXX + t1; idx[8] = FXX + t2; idx[9] = mixed_of(t1, t2);
}

/* map ghost index j along an axis of n cells: returns the source cell and
   sets *flip = -1 when reached through an odd number of reflections */
static int bc_map(int j, int n, int bc, double *flip)
{
    *flip = 1.0;
    if (bc == 0) return ((j % n) + n) % n;
    int p = 2 * n;
    int k = ((j % p) + p) % p;
    if (k < n) return k;
    *flip = -1.0;
    return p - 1 - k;
}

static void compute_flattening(or_sim *S, int d);

static void do_pass(or_sim *S, int d, double dt)
{
    const or_params *P = &S->P;
    const int n = P->n[d];
    if (S->flat_on) compute_flattening(S, d);   /* of this pass's input */
    const int a1 = (d + 1) % 3, a2 = (d + 2) % 3;    /* transverse axes */
    const int na1 = P->n[a1], na2 = P->n[a2];
    int pidx[10];
    ppb_order(d, pidx);
    const int odd_ppb[10] = { 0, 1, 0, 0, 1, 0, 1, 0, 0, 0 };
    unsigned long long unsm = 0, ncv = 0, hits = 0;

    #pragma omp parallel num_threads(S->nthreads) reduction(+:unsm,ncv,hits)
    {
        pencil pc;
        pencil_alloc(&pc, n);
        #pragma omp for schedule(static)
        for (long pe = 0; pe < (long)na1 * na2; ++pe) {
            int t1 = (int)(pe % na1), t2 = (int)(pe / na1);
            pc.unsmooth = pc.nonconv = pc.hits = 0;
            pc.diss_k = S->diss_k;
            pc.flat_on = S->flat_on;
            for (int j = -NG; j < n + NG; ++j) {
                int J = j + NG;
                double fl;
                int s = bc_map(j, n, P->bc[d], &fl);
                int ijk[3];
                ijk[d] = s; ijk[a1] = t1; ijk[a2] = t2;
                long ci = cidx(S, ijk[0], ijk[1], ijk[2]);
                double x[3], gv[3];
                cell_pos(P, ijk[0], ijk[1], ijk[2], x);
                gravity_at(P, x, gv);
                pc.rhop[J] = S->U[RHO][ci];
                pc.mn[J] = fl * S->U[MX + d][ci];
                pc.mt1[J] = S->U[MX + a1][ci];
                pc.mt2[J] = S->U[MX + a2][ci];
                pc.ep[J] = S->U[EN][ci];
                pc.r0[J] = S->rho0[ci];
                pc.p0[J] = S->p0[ci];
                pc.g[J] = fl * gv[d];
                pc.solid[J] = solid_at(P, x);
                pc.div[J] = S->diss_k > 0.0 ? S->divu[ci] : 0.0;
                pc.flat[J] = S->flat_on ? S->flat[ci] : 0.0;
                for (int q = 0; q < 10; ++q)
                    pc.f[q][J] = (odd_ppb[q] ? fl : 1.0) * S->U[pidx[q]][ci];
            }
            pencil_update(&pc, dt, P->dx, P->gamma, P->smooth_detect);
            for (int j = 0; j < n; ++j) {
                int J = j + NG;
                int ijk[3];
                ijk[d] = j; ijk[a1] = t1; ijk[a2] = t2;
                long ci = cidx(S, ijk[0], ijk[1], ijk[2]);
                S->W[RHO][ci] = pc.o_rhop[J];
                S->W[MX + d][ci] = pc.o_mn[J];
                S->W[MX + a1][ci] = pc.o_mt1[J];
                S->W[MX + a2][ci] = pc.o_mt2[J];
                S->W[EN][ci] = pc.o_ep[J];
                for (int q = 0; q < 10; ++q) S->W[pidx[q]][ci] = pc.o_f[q][J];
            }
            unsm += pc.unsmooth; ncv += pc.nonconv; hits += pc.hits;
        }
        pencil_free(&pc);
    }
    for (int q = 0; q < NF; ++q) { double *t = S->U[q]; S->U[q] = S->W[q]; S->W[q] = t; }
    S->cnt[0] += hits; S->cnt[1] += unsm; S->cnt[2] += ncv;
}

/* ------------------------------------------------------------------ */
/* Public entry points (ctypes)                                          */
/* ------------------------------------------------------------------ */

void *or_create(const or_params *P, int nthreads)
{
    or_sim *S = (or_sim *)calloc(1, sizeof(or_sim));
    S->P = *P;
    S->ncell = (long)P->n[0] * P->n[1] * P->n[2];
    S->nthreads = nthreads > 0 ? nthreads : 1;
    for (int q = 0; q < NF; ++q) {
        S->U[q] = (double *)calloc(S->ncell, sizeof(double));
        S->W[q] = (double *)calloc(S->ncell, sizeof(double));
        if (!S->U[q] || !S->W[q]) return NULL;
    }
    S->rho0 = (double *)calloc(S->ncell, sizeof(double));
    S->p0 = (double *)calloc(S->ncell, sizeof(double));
    base_fill(S);
    return S;
}

void or_destroy(void *h)
{
    or_sim *S = (or_sim *)h;
    if (!S) return;
    for (int q = 0; q < NF; ++q) { free(S->U[q]); free(S->W[q]); }
    free(S->rho0); free(S->p0); free(S->divu); free(S->flat); free(S);
}

void or_set_threads(void *h, int nthreads) { ((or_sim *)h)->nthreads = nthreads > 0 ? nthreads : 1; }

/* Set the state from perturbation primitives (rho', u, v, w, p') and the
   10 fv coefficients: m = rho u, E' = p'/(gamma-1) + rho |u|^2 / 2. */
void or_set_state(void *h, double *const *prim)
{
    or_sim *S = (or_sim *)h;
    double gm1 = S->P.gamma - 1.0;
    for (long c = 0; c < S->ncell; ++c) {
        double rho = S->rho0[c] + prim[0][c];
        double u = prim[1][c], v = prim[2][c], w = prim[3][c];
        S->U[RHO][c] = prim[0][c];
        S->U[MX][c] = rho * u; S->U[MY][c] = rho * v; S->U[MZ][c] = rho * w;
        S->U[EN][c] = prim[4][c] / gm1 + 0.5 * rho * ((u * u + v * v) + w * w);
        for (int q = 0; q < 10; ++q) S->U[F0 + q][c] = prim[5 + q][c];
    }
}

void or_get_state(void *h, double *const *prim)
{
    or_sim *S = (or_sim *)h;
    double gm1 = S->P.gamma - 1.0;
    for (long c = 0; c < S->ncell; ++c) {
        double rho = S->rho0[c] + S->U[RHO][c];
        double u = S->U[MX][c] / rho, v = S->U[MY][c] / rho, w = S->U[MZ][c] / rho;
        prim[0][c] = S->U[RHO][c];
        prim[1][c] = u; prim[2][c] = v; prim[3][c] = w;
        prim[4][c] = gm1 * (S->U[EN][c] - 0.5 * (S->U[MX][c] * u + S->U[MY][c] * v + S->U[MZ][c] * w));
        for (int q = 0; q < 10; ++q) prim[5 + q][c] = S->U[F0 + q][c];
    }
}

void or_get_conserved(void *h, double *const *cons)
{
    or_sim *S = (or_sim *)h;
    for (int q = 0; q < NF; ++q) memcpy(cons[q], S->U[q], sizeof(double) * S->ncell);
}

void or_set_conserved(void *h, double *const *cons)
{
    or_sim *S = (or_sim *)h;
    for (int q = 0; q < NF; ++q) memcpy(S->U[q], cons[q], sizeof(double) * S->ncell);
}

void or_get_base(void *h, double *rho0, double *p0)
{
    or_sim *S = (or_sim *)h;
    memcpy(rho0, S->rho0, sizeof(double) * S->ncell);
    memcpy(p0, S->p0, sizeof(double) * S->ncell);
}

/* base profile at arbitrary coordinates, for the closed-form pin */
void or_base_profile(const or_params *P, int npts, const double *s, double *rho, double *p)
{
    base_table T;
    base_build(P, &T);
    for (int q = 0; q < npts; ++q) base_eval(P, &T, s[q], &rho[q], &p[q]);
    base_free(&T);
}

/* CFL time step: dt = cfl dx / max over fluid cells of max_d |u_d| + c.
   The maximum does not depend on the order of evaluation. */
double or_compute_dt(void *h, double cfl)
{
    or_sim *S = (or_sim *)h;
    const or_params *P = &S->P;
    double gm1 = P->gamma - 1.0, smax = 0.0;
    for (int k = 0; k < P->n[2]; ++k)
        for (int j = 0; j < P->n[1]; ++j)
            for (int i = 0; i < P->n[0]; ++i) {
                double x[3];
                cell_pos(P, i, j, k, x);
                if (solid_at(P, x)) continue;
                long c = cidx(S, i, j, k);
                double rho = S->rho0[c] + S->U[RHO][c];
                double u = S->U[MX][c] / rho, v = S->U[MY][c] / rho, w = S->U[MZ][c] / rho;
                double pp = gm1 * (S->U[EN][c] - 0.5 * (S->U[MX][c] * u + S->U[MY][c] * v + S->U[MZ][c] * w));
                double cs = sqrt(P->gamma * (S->p0[c] + pp) / rho);
                double s = fmax(fabs(u), fmax(fabs(v), fabs(w))) + cs;
                if (s > smax) smax = s;
            }
    return cfl * P->dx / smax;
}

/* ------------------------------------------------------------------ */
/* Rotation and shell averages (Sec. 1, Sec. 3)                          */
/* ------------------------------------------------------------------ */

/* Spin-up (Sec. 3: a solid-body rotational flow is added gradually over
   the first steps of a run, in the inertial frame).  [reading] Every fluid
   cell gets the velocity increment domega * (z-hat x x) = domega * (-y, x, 0)
   at its centre, the density and the pressure perturbation are left as they
   are; m and E' are rebuilt from the new velocity. */
void or_spin_add(void *h, double domega)
{
    or_sim *S = (or_sim *)h;
    const or_params *P = &S->P;
    double gm1 = P->gamma - 1.0;
    for (int k = 0; k < P->n[2]; ++k)
        for (int j = 0; j < P->n[1]; ++j)
            for (int i = 0; i < P->n[0]; ++i) {
                double x[3];
                cell_pos(P, i, j, k, x);
                if (solid_at(P, x)) continue;
                long c = cidx(S, i, j, k);
                double rho = S->rho0[c] + S->U[RHO][c];
                double u = S->U[MX][c] / rho, v = S->U[MY][c] / rho, w = S->U[MZ][c] / rho;
                double pp = gm1 * (S->U[EN][c] - 0.5 * (S->U[MX][c] * u + S->U[MY][c] * v + S->U[MZ][c] * w));
                u += -domega * x[1];
                v += domega * x[0];
                S->U[MX][c] = rho * u;
                S->U[MY][c] = rho * v;
                S->U[EN][c] = pp / gm1 + 0.5 * rho * ((u * u + v * v) + w * w);
            }
}

/* Rotating frame (Sec. 3: the runs keep the inertial frame and name
   rotating coordinates as the next step).  [reading] Axes turning at omega
   about the z axis through the coordinate origin add two accelerations to
   the momentum equation: the Coriolis term -2 omega z-hat x u =
   2 omega (u_y, -u_x, 0) and, when `centrifugal` is set, the centrifugal
   term omega^2 (x, y, 0).  Each step ends, after the passes and the
   heating, with these sources over dt as a split step of its own, in three
   parts: half the centrifugal velocity change omega^2 (x, y) dt / 2; then
   the exact solution of the Coriolis part alone over dt, which turns
   (u_x, u_y) by the angle -2 omega dt; then the other half of the
   centrifugal change.  Density and pressure are kept; m and E' are rebuilt
   from the new velocity.  Solid cells are not touched. */
static void rotframe(or_sim *S, double dt)
{
    const or_params *P = &S->P;
    const double om = S->rot_omega, gm1 = P->gamma - 1.0;
    const double th = -2.0 * om * dt, cth = cos(th), sth = sin(th);
    const double kick = S->rot_centrifugal ? 0.5 * om * om * dt : 0.0;
    for (int k = 0; k < P->n[2]; ++k)
        for (int j = 0; j < P->n[1]; ++j)
            for (int i = 0; i < P->n[0]; ++i) {
                double x[3];
                cell_pos(P, i, j, k, x);
                if (solid_at(P, x)) continue;
                long c = cidx(S, i, j, k);
                double rho = S->rho0[c] + S->U[RHO][c];
                double u = S->U[MX][c] / rho, v = S->U[MY][c] / rho, w = S->U[MZ][c] / rho;
                double pp = gm1 * (S->U[EN][c] - 0.5 * (S->U[MX][c] * u + S->U[MY][c] * v + S->U[MZ][c] * w));
                u += kick * x[0];
                v += kick * x[1];
                double ur = cth * u - sth * v, vr = sth * u + cth * v;
                u = ur + kick * x[0];
                v = vr + kick * x[1];
                S->U[MX][c] = rho * u;
                S->U[MY][c] = rho * v;
                S->U[EN][c] = pp / gm1 + 0.5 * rho * ((u * u + v * v) + w * w);
            }
}

void or_set_rotating_frame(void *h, double omega, int centrifugal)
{
    or_sim *S = (or_sim *)h;
    S->rot_omega = omega;
    S->rot_centrifugal = centrifugal ? 1 : 0;
}

/* Ramp: the steps with index 0 .. nramp-1 each end with an increment of
   omega / nramp, so that the rotation reaches omega after nramp steps.
   nramp <= 0 or omega == 0 switches the ramp off. */
void or_set_spinup(void *h, double omega, long nramp)
{
    or_sim *S = (or_sim *)h;
    S->spin_omega = omega;
    S->spin_nramp = (omega != 0.0 && nramp > 0) ? nramp : 0;
}

/* Averages on spherical surfaces (Sec. 1: the runs produce averages over
   spheres that inform 1-D models).  Shell k holds the fluid cells whose
   centre radius r (from the coordinate origin) has (k dr)^2 <= r^2 <
   ((k+1) dr)^2, all in FP64 with r^2 = (x^2 + y^2) + z^2.  Per shell,
   out[8k + q] is the sum over its cells of dV times
     q = 0: 1            (volume)
         1: rho          (mass)
         2: fv           (entrained-fluid volume)
         3: rho u_r      (radial mass flux; u_r = x.u / r)
         4: rho u_r^2
         5: rho |u|^2
         6: rho (x v - y u)  (angular momentum about z)
         7: fv^2
   so that volume-weighted and mass-weighted shell averages are ratios. */
void or_shell_profile(void *h, int nbins, double dr, double *out)
{
    or_sim *S = (or_sim *)h;
    const or_params *P = &S->P;
    double dv = P->dx * P->dx * P->dx;
    double rmax2 = ((double)nbins * dr) * ((double)nbins * dr);
    for (long q = 0; q < 8L * nbins; ++q) out[q] = 0.0;
    for (int k = 0; k < P->n[2]; ++k)
        for (int j = 0; j < P->n[1]; ++j)
            for (int i = 0; i < P->n[0]; ++i) {
                double x[3];
                cell_pos(P, i, j, k, x);
                if (solid_at(P, x)) continue;
                double r2 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
                if (!(r2 < rmax2)) continue;
                /* shell index from the squared bounds */
                int b = (int)(sqrt(r2) / dr);
                if (b > nbins - 1) b = nbins - 1;
                while (b > 0 && ((double)b * dr) * ((double)b * dr) > r2) --b;
                while (b < nbins - 1 && ((double)(b + 1) * dr) * ((double)(b + 1) * dr) <= r2) ++b;
                long c = cidx(S, i, j, k);
                double rho = S->rho0[c] + S->U[RHO][c];
                double u = S->U[MX][c] / rho, v = S->U[MY][c] / rho, w = S->U[MZ][c] / rho;
                double r = sqrt(r2);
                double ur = r > 0.0 ? (x[0] * u + x[1] * v + x[2] * w) / r : 0.0;
                double f = S->U[F0][c];
                double *o = out + 8L * b;
                o[0] += dv;
                o[1] += rho * dv;
                o[2] += f * dv;
                o[3] += rho * ur * dv;
                o[4] += rho * ur * ur * dv;
                o[5] += rho * ((u * u + v * v) + w * w) * dv;
                o[6] += rho * (x[0] * v - x[1] * u) * dv;
                o[7] += f * f * dv;
            }
}

/* Shock dissipation (Sec. 1: a fully 3-D dissipation inside shocks; its
   form is in a reference that is not available).  [reading] The undivided
   divergence of the cell-centred velocity, D = sum over d of
   (u_d(i + e_d) - u_d(i - e_d)) / 2, with the boundary images of the
   neighbours (a solid neighbour is a wall: its normal velocity is minus
   the cell's own), taken once at the start of a step; each pass adds at a
   face between fluid cells the flux K max(0, -(D_i + D_i+1)/2) (U_i - U_i+1)
   to the five conserved hydro perturbations.  Zero wherever the flow does
   not converge, conservative, and along every axis driven by the same 3-D
   compression. */
static double cell_velocity(const or_sim *S, long c, int d)
{
    double rho = S->rho0[c] + S->U[RHO][c];
    return S->U[MX + d][c] / rho;
}

static void compute_divergence(or_sim *S)
{
    const or_params *P = &S->P;
    if (!S->divu) S->divu = (double *)calloc(S->ncell, sizeof(double));
    for (int k = 0; k < P->n[2]; ++k)
        for (int j = 0; j < P->n[1]; ++j)
            for (int i = 0; i < P->n[0]; ++i) {
                double x[3];
                cell_pos(P, i, j, k, x);
                long c = cidx(S, i, j, k);
                if (solid_at(P, x)) { S->divu[c] = 0.0; continue; }
                double D = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double un[2];
                    for (int side = 0; side < 2; ++side) {
                        int ijk[3] = { i, j, k };
                        double fl;
                        ijk[d] = bc_map(ijk[d] + (side ? 1 : -1), P->n[d], P->bc[d], &fl);
                        double xn[3];
                        cell_pos(P, ijk[0], ijk[1], ijk[2], xn);
                        if (solid_at(P, xn)) un[side] = -cell_velocity(S, c, d);
                        else un[side] = fl * cell_velocity(S, cidx(S, ijk[0], ijk[1], ijk[2]), d);
                    }
                    D += 0.5 * (un[1] - un[0]);
                }
                S->divu[c] = D;
            }
}

void or_set_dissipation(void *h, double k) { ((or_sim *)h)->diss_k = k > 0.0 ? k : 0.0; }

/* Flattening near strong shocks, after Colella & Woodward (1984, Sec. 4)
   [reading: the paper names only the 3-D shock dissipation; flattening is
   CW84's companion device, with their constants].  For the pass along d,
   with p the full pressure and u the velocity along d (neighbours through
   the boundary conditions, a reflecting image's u flipped):
     a cell is a shock candidate when |p(+1) - p(-1)| > eps min(p(+1), p(-1))
     and the flow converges, u(-1) - u(+1) > tie (|u(-1)| + |u(+1)|);
     its raw coefficient is min(1, max(0, w2 (z - w1))) with
     z = (p(+1) - p(-1)) / (p(+2) - p(-2)) (0 where the wide difference is
     0), and 0 for a cell that is no candidate;
     its coefficient is the larger of its own raw value and that of its
     neighbour on the low-pressure side (+1 when p(+1) < p(-1), else -1),
     or of both neighbours when |p(+1) - p(-1)| <= tie (p(+1) + p(-1)).
   The two tie margins [reading: CW84's tests are strict] keep decisions
   off values that are equal but for rounding (a uniform transverse flow
   after a pass gives neighbours the same velocity to the last bit or two),
   where a strict test would switch the flattening on or off at random; a
   real shock lies orders of magnitude above them.  The symmetric tie rule
   also keeps the coefficient mirror symmetric. */
#define FLAT_EPS 0.33
#define FLAT_W1 0.75
#define FLAT_W2 10.0
#define FLAT_TIE 1e-10

static double cell_pressure(const or_sim *S, long c)
{
    double rho = S->rho0[c] + S->U[RHO][c];
    double mx = S->U[MX][c], my = S->U[MY][c], mz = S->U[MZ][c];
    double pp = (S->P.gamma - 1.0) * (S->U[EN][c] - 0.5 * (mx * (mx / rho) + my * (my / rho) + mz * (mz / rho)));
    return S->p0[c] + pp;
}

static double flat_raw(const double *p, const double *u, int o)
{
    /* p, u indexed by offset + 3 */
    double dp1 = p[o + 4] - p[o + 2], dp2 = p[o + 5] - p[o + 1];
    int cand = fabs(dp1) > FLAT_EPS * fmin(p[o + 4], p[o + 2]) &&
               u[o + 2] - u[o + 4] > FLAT_TIE * (fabs(u[o + 2]) + fabs(u[o + 4]));
    if (!cand) return 0.0;
    double z = dp2 != 0.0 ? dp1 / dp2 : 0.0;
    return fmin(1.0, fmax(0.0, FLAT_W2 * (z - FLAT_W1)));
}

static void compute_flattening(or_sim *S, int d)
{
    const or_params *P = &S->P;
    if (!S->flat) S->flat = (double *)calloc(S->ncell, sizeof(double));
    #pragma omp parallel for num_threads(S->nthreads) schedule(static)
    for (long c = 0; c < S->ncell; ++c) {
        int ijk[3] = { (int)(c % P->n[0]), (int)((c / P->n[0]) % P->n[1]), (int)(c / ((long)P->n[0] * P->n[1])) };
        double p[7], u[7];
        for (int o = -3; o <= 3; ++o) {
            int nb[3] = { ijk[0], ijk[1], ijk[2] };
            double fl;
            nb[d] = bc_map(ijk[d] + o, P->n[d], P->bc[d], &fl);
            long e = cidx(S, nb[0], nb[1], nb[2]);
            p[o + 3] = cell_pressure(S, e);
            u[o + 3] = fl * cell_velocity(S, e, d);
        }
        double f0 = flat_raw(p, u, 0), fm = flat_raw(p, u, -1), fp = flat_raw(p, u, 1);
        double dp = p[4] - p[2];
        double nb;
        if (fabs(dp) <= FLAT_TIE * (p[4] + p[2])) nb = fmax(fm, fp);
        else nb = dp < 0.0 ? fp : fm;
        S->flat[c] = fmax(f0, nb);
    }
}

void or_set_flattening(void *h, int on) { ((or_sim *)h)->flat_on = on ? 1 : 0; }

/* Gravity and heating changed during a run (Sec. 3 gravity, Sec. 2 heating):
   the parameters of the following passes; the base state is kept as it is. */
void or_set_gravity(void *h, int kind, const double g[4])
{
    or_sim *S = (or_sim *)h;
    S->P.grav_kind = kind;
    for (int q = 0; q < 4; ++q) S->P.grav[q] = g[q];
}

void or_set_heating(void *h, int kind, const double q3[3])
{
    or_sim *S = (or_sim *)h;
    S->P.heat_kind = kind;
    for (int q = 0; q < 3; ++q) S->P.heat[q] = q3[q];
}

/* the flattening coefficients of the current state for a pass along d */
void or_flattening(void *h, int d, double *out)
{
    or_sim *S = (or_sim *)h;
    compute_flattening(S, d);
    memcpy(out, S->flat, sizeof(double) * S->ncell);
}

/* the divergence field of the current state (cells x fastest) */
void or_divergence(void *h, double *out)
{
    or_sim *S = (or_sim *)h;
    compute_divergence(S);
    memcpy(out, S->divu, sizeof(double) * S->ncell);
}

/* One pass on its own: with dissipation on, from the divergence of its
   input state. */
void or_pass(void *h, int axis, double dt)
{
    or_sim *S = (or_sim *)h;
    if (S->diss_k > 0.0) compute_divergence(S);
    do_pass(S, axis, dt);
}

/* One step: three passes, x,y,z on even steps and z,y,x on odd ones
   [reading: the paper only says three 1-D passes], then the heating source,
   then, during a spin-up ramp, the rotation increment. */
void or_step(void *h, double dt)
{
    or_sim *S = (or_sim *)h;
    const or_params *P = &S->P;
    if (S->diss_k > 0.0) compute_divergence(S);
    if (S->nstep % 2 == 0) { do_pass(S, 0, dt); do_pass(S, 1, dt); do_pass(S, 2, dt); }
    else                   { do_pass(S, 2, dt); do_pass(S, 1, dt); do_pass(S, 0, dt); }
    if (P->heat_kind != 0) {
        for (int k = 0; k < P->n[2]; ++k)
            for (int j = 0; j < P->n[1]; ++j)
                for (int i = 0; i < P->n[0]; ++i) {
                    double x[3];
                    cell_pos(P, i, j, k, x);
                    if (solid_at(P, x)) continue;
                    S->U[EN][cidx(S, i, j, k)] += heating_at(P, x) * dt;
                }
    }
    if (S->rot_omega != 0.0) rotframe(S, dt);
    if (S->nstep < S->spin_nramp) or_spin_add(h, S->spin_omega / (double)S->spin_nramp);
    S->nstep++;
    S->cnt[3]++;
}

long or_nstep(void *h) { return ((or_sim *)h)->nstep; }
void or_set_nstep(void *h, long n) { ((or_sim *)h)->nstep = n; }

static double pairwise_sum(const double *a, long n)
{
    if (n <= 8) { double s = 0.0; for (long i = 0; i < n; ++i) s += a[i]; return s; }
    long h = n / 2;
    return pairwise_sum(a, h) + pairwise_sum(a + h, n - h);
}

/* Conserved totals over fluid cells: mass, momentum, total energy (base
   included), fv volume, and min / max of the fv average. */
void or_totals(void *h, double out[8])
{
    or_sim *S = (or_sim *)h;
    const or_params *P = &S->P;
    double dv = P->dx * P->dx * P->dx, gm1 = P->gamma - 1.0;
    double *buf = (double *)malloc(sizeof(double) * S->ncell);
    double fmn = INFINITY, fmx = -INFINITY;
    for (int q = 0; q < 6; ++q) {
        for (int k = 0; k < P->n[2]; ++k)
            for (int j = 0; j < P->n[1]; ++j)
                for (int i = 0; i < P->n[0]; ++i) {
                    double x[3];
                    cell_pos(P, i, j, k, x);
                    long c = cidx(S, i, j, k);
                    double val = 0.0;
                    if (!solid_at(P, x)) {
                        switch (q) {
                        case 0: val = S->rho0[c] + S->U[RHO][c]; break;
                        case 1: val = S->U[MX][c]; break;
                        case 2: val = S->U[MY][c]; break;
                        case 3: val = S->U[MZ][c]; break;
                        case 4: val = S->p0[c] / gm1 + S->U[EN][c]; break;
                        case 5: val = S->U[F0][c];
                                if (val < fmn) fmn = val;
                                if (val > fmx) fmx = val;
                                break;
                        }
                    }
                    buf[c] = val;
                }
        out[q] = pairwise_sum(buf, S->ncell) * dv;
    }
    out[6] = fmn; out[7] = fmx;
    free(buf);
}

void or_counters(void *h, unsigned long long out[4])
{
    or_sim *S = (or_sim *)h;
    for (int q = 0; q < 4; ++q) out[q] = S->cnt[q];
}

int or_sizeof_params(void) { return (int)sizeof(or_params); }
