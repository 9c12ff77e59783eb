/*
 * oracle.c -- plain, slow FP64 CPU reference for the explicit finite-volume
 * discrete-velocity (DVM) time step of the Shakhov model with ghost-cell
 * immersed boundaries (Ge, Cai, Zhang, Xiao, "An immersed boundary method for
 * the discrete velocity model of the Boltzmann equation", arXiv 2512.20252).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it is used by tests/, by the smoke check and by the CPU
 * baseline leg of the benchmark.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Every sum over velocity nodes runs sequentially in node order; there is no
 * blocking, fusion or reordering.  Each function names the passage of the
 * paper it follows.  Where the paper is silent or garbled, the reading used is
 * stated next to the code (R-numbers refer to the list of readings kept with
 * the design notes).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 *
 * Layout: cell c = i + n0*(j + n1*l) (x fastest); velocity node
 * k = ix + N0*(iy + N1*iz); distributions f[A][c*NV + k].  In 2D the two
 * arrays are the reduced distributions h (A=0) and b (A=1) (Section 4,
 * reduced distributions); in 3D there is one array f.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_FREESTREAM 0
#define OR_PERIODIC 1
#define OR_WALLS 2 /* 2D: diffuse walls on all four sides, the side y = hi moving along x */
/* 2D: specular walls on all four sides (reading R32) */
#define OR_SPECULAR 3

#define OR_G_NONE 0
#define OR_G_CIRCLE 1
#define OR_G_ELLIPSE 2
#define OR_G_AIRFOIL 3
#define OR_G_SPHERE 4

#define OR_RULE_MIDPOINT 0
#define OR_RULE_TRAPEZOID 1
/* stretched tensor grid (reading R31): the midpoint grid of u in [-1, 1]
 * mapped by x(u) = V sinh(beta u) / sinh(beta), finer near xi = 0 */
#define OR_RULE_STRETCHED 2
/* locally refined tensor grid (reading R35): per axis the node density
 * 1 + A (exp(-(x/w)^2) + exp(-((x - c)/w)^2)) (one bump when c = 0),
 * nodes and dual cells the images of the uniform u-cells under the inverse
 * of its normalised cumulative */
#define OR_RULE_REFINED 3

/* node weights of the mapped grids (stretched and refined): the width of
 * the node's dual cell, or (reading R36) the derivative of the map at the
 * node times the width of its u-cell, the midpoint rule of the integral
 * in u; cut cells keep their incident fraction of the dual cell */
#define OR_WEIGHTS_CELL 0
#define OR_WEIGHTS_JACOBIAN 1

#define OR_FLAG_NO_CUTCELL 1u
#define OR_FLAG_NO_UPWIND 2u
/* semi-implicit collision (reading R30): explicit transport, then the
 * Shakhov relaxation taken implicitly with the moments of the transported
 * state */
#define OR_FLAG_IMPLICIT 4u
/* reading R28(2) as an option: the ghost-side face value is taken on the
 * shifted-point -> wall line no further than the wall */
#define OR_FLAG_FACE_LIMIT 8u
/* ablation of Section 3.3.3: the intermediate ghost value is the naive
 * linear extrapolation of donor and auxiliary cell along the pair's axis
 * instead of the upwind-weighted surface-cell interpolation */
#define OR_FLAG_NAIVE 16u
/* ablation: no donor slope (reading R10 on every pair), the shifted-point
 * value is the donor value */
#define OR_FLAG_NO_AUX 32u

/* velocity-node classes of one pair (Section 3.2.3): fully incident ("gas"),
 * fully reflected ("solid"), cut with node on the incident side (set G) and
 * cut with node on the reflected side (set S). */
#define CL_GAS 0
#define CL_SOLID 1
#define CL_CUT_G 2
#define CL_CUT_S 3

typedef struct {
    int dim;
    int n[3];
    double lo[3], hi[3];
    int outer;
    int vn[3];
    double vlo[3], vhi[3];
    int vrule;
    int gkind;
    double gcen[3];
    double gsize[3];
    double aoa;
    double Kn, Ma, Pr, gam, alpha, Tw, cfl, omega, avhs;
    int flags;
    double lid_u; /* OR_WALLS: velocity of the wall at y = hi, along x */
    double vstretch; /* OR_RULE_STRETCHED: beta */
    /* body wall velocity at the wall point x_w: Uw + Ow x (x_w - centre),
     * a translation plus a rigid rotation about the geometry centre (in 2D
     * only Ow[2] acts); the wall Maxwellian of Section 2.3 moves with it */
    double Uw[3], Ow[3];
    /* OR_RULE_REFINED: amplitude A, width w and second centre c per axis */
    double vref_amp, vref_width, vref_centre[3];
    int vweights; /* OR_WEIGHTS_*: mapped grids only */
} or_case;

typedef struct {
    int gc, dc, ac; /* ghost, donor, auxiliary cell (ac = -1: none) */
    int axis, sign; /* dc = gc + sign * e_axis */
    double xw[3], nw[3], xsp[3];
    double uw[3]; /* wall velocity at x_w */
    int ns;
    int sc[26];
    double r[26][3], rh[26][3];
    unsigned char *cls; /* [NV] */
    double *wg;         /* [NV] incident-side measure of the dual cell */
} or_pair;

typedef struct {
    or_case c;
    int D, Nc, NV, NA;
    double dx[3];
    double *xi1[3], *w1[3];
    double *ed0[3], *ed1[3]; /* dual cell [ed0, ed1] of each node per axis */
    double dxi[3];
    double *xi;   /* [NV*3] */
    double *w;    /* [NV] */
    double maxabs[3];
    unsigned char *solid; /* [Nc] */
    int *pnb;             /* [Nc*6]: pair seen from fluid cell c in direction (axis, side) */
    int npairs;
    or_pair *pairs;
    int nghost;
    double *f[2], *fn[2];
    double *fs[2]; /* freestream distributions [NV] */
    double *mom;   /* [Nc*8] rho, U0..U2, T, q0..q2 */
    double *tau;   /* [Nc] */
    double mu0;
    double dt, time;
    long step;
    /* per-pair work arrays [npairs*NV] */
    double *fsp[2], *fgc[2], *fiw[2], *fss[2], *fw[2], *gh[2], *fc[2];
    double *rhow; /* [npairs] */
    double Uinf;
    /* OR_WALLS: ghost rows of the boundary cells, sides x-, x+, y-, y+ in
     * turn, one row per boundary cell along the wall [2 (nx + ny)][NV] */
    double *wgh[2];
} or_state;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static double xc(const or_state *s, int a, int i) { return s->c.lo[a] + ((double)i + 0.5) * s->dx[a]; }

static void cell_ijk(const or_state *s, int c, int ijk[3])
{
    ijk[0] = c % s->c.n[0];
    ijk[1] = (c / s->c.n[0]) % s->c.n[1];
    ijk[2] = (s->D == 3) ? c / (s->c.n[0] * s->c.n[1]) : 0;
}

static int cell_id(const or_state *s, const int ijk[3])
{
    return ijk[0] + s->c.n[0] * (ijk[1] + s->c.n[1] * (s->D == 3 ? ijk[2] : 0));
}

static int in_grid(const or_state *s, const int ijk[3])
{
    for (int a = 0; a < s->D; ++a)
        if (ijk[a] < 0 || ijk[a] >= s->c.n[a]) return 0;
    return 1;
}

/* van Leer limited slope as printed in Section 2.2 (limiter equation):
 * (sign s1 + sign s2) |s1||s2| / (|s1| + |s2|), zero when both vanish. */
static double vanleer(double s1, double s2)
{
    double sg1 = (s1 > 0) - (s1 < 0), sg2 = (s2 > 0) - (s2 < 0);
    double den = fabs(s1) + fabs(s2);
    if (den == 0.0) return 0.0;
    return (sg1 + sg2) * fabs(s1) * fabs(s2) / den;
}

/* ------------------------------------------------------------------ */
/* geometry: level sets (negative inside the solid)                    */
/* ------------------------------------------------------------------ */

static double naca_yt(double t, double X)
{
    /* symmetric 4-digit half thickness, closed trailing edge (reading R19) */
    return 5.0 * t * (0.2969 * sqrt(X) - 0.1260 * X - 0.3516 * X * X + 0.2843 * X * X * X - 0.1036 * X * X * X * X);
}

static double naca_dyt(double t, double X)
{
    if (X < 1e-12) X = 1e-12;
    return 5.0 * t * (0.2969 * 0.5 / sqrt(X) - 0.1260 - 2.0 * 0.3516 * X + 3.0 * 0.2843 * X * X - 4.0 * 0.1036 * X * X * X);
}

static void body_frame(const or_case *c, const double x[3], double *xp, double *yp)
{
    double dx = x[0] - c->gcen[0], dy = x[1] - c->gcen[1];
    double ca = cos(c->aoa), sa = sin(c->aoa);
    *xp = dx * ca - dy * sa;
    *yp = dx * sa + dy * ca;
}

static double phi(const or_state *s, const double x[3])
{
    const or_case *c = &s->c;
    switch (c->gkind) {
    case OR_G_CIRCLE: {
        double dx = x[0] - c->gcen[0], dy = x[1] - c->gcen[1];
        return dx * dx + dy * dy - c->gsize[0] * c->gsize[0];
    }
    case OR_G_SPHERE: {
        double dx = x[0] - c->gcen[0], dy = x[1] - c->gcen[1], dz = x[2] - c->gcen[2];
        return dx * dx + dy * dy + dz * dz - c->gsize[0] * c->gsize[0];
    }
    case OR_G_ELLIPSE: {
        double xp, yp;
        body_frame(c, x, &xp, &yp);
        double u = xp / c->gsize[0], v = yp / c->gsize[1];
        return u * u + v * v - 1.0;
    }
    case OR_G_AIRFOIL: {
        double xp, yp;
        body_frame(c, x, &xp, &yp);
        double ch = c->gsize[0];
        double X = xp / ch, Y = yp / ch;
        if (X < 0.0) return ch * sqrt(X * X + Y * Y);
        if (X > 1.0) return ch * sqrt((X - 1.0) * (X - 1.0) + Y * Y);
        return ch * (fabs(Y) - naca_yt(c->gsize[1], X));
    }
    default:
        return 1.0;
    }
}

/* unit normal grad(phi)/|grad(phi)|, pointing from the solid into the gas */
static void normal(const or_state *s, const double x[3], double nrm[3])
{
    const or_case *c = &s->c;
    double g[3] = {0, 0, 0};
    switch (c->gkind) {
    case OR_G_CIRCLE:
    case OR_G_SPHERE:
        for (int a = 0; a < s->D; ++a) g[a] = 2.0 * (x[a] - c->gcen[a]);
        break;
    case OR_G_ELLIPSE:
    case OR_G_AIRFOIL: {
        double xp, yp, gx, gy;
        body_frame(c, x, &xp, &yp);
        if (c->gkind == OR_G_ELLIPSE) {
            gx = 2.0 * xp / (c->gsize[0] * c->gsize[0]);
            gy = 2.0 * yp / (c->gsize[1] * c->gsize[1]);
        } else {
            double ch = c->gsize[0];
            double X = xp / ch, Y = yp / ch;
            if (X <= 0.0) {
                gx = X;
                gy = Y;
            } else if (X >= 1.0) {
                gx = X - 1.0;
                gy = Y;
            } else {
                gx = -naca_dyt(c->gsize[1], X);
                gy = (Y >= 0.0) ? 1.0 : -1.0;
            }
        }
        double ca = cos(c->aoa), sa = sin(c->aoa);
        /* x' = d.e1, y' = d.e2 with e1 = (cos, -sin), e2 = (sin, cos) */
        g[0] = gx * ca + gy * sa;
        g[1] = -gx * sa + gy * ca;
        break;
    }
    default:
        g[0] = 1.0;
    }
    double m = 0.0;
    for (int a = 0; a < s->D; ++a) m += g[a] * g[a];
    m = sqrt(m);
    for (int a = 0; a < 3; ++a) nrm[a] = (a < s->D) ? g[a] / m : 0.0;
}

/* ------------------------------------------------------------------ */
/* velocity space (Section 2.2 quadrature; midpoint rule of 3.2.3)     */
/* ------------------------------------------------------------------ */

/* stretched map of reading R31 at u = m / N (m an integer in [-N, N], so
 * that -m gives exactly the negated value) */
static double stretch_map(double V, double beta, int m, int N)
{
    return V * sinh(beta * ((double)m / (double)N)) / sinh(beta);
}

/* cumulative node density of the refined rule (reading R35) from -V to x:
 * the integral of 1 + A sum_c exp(-((x - c)/w)^2), each bump integrating
 * to A w sqrt(pi)/2 (erf(.) - erf(.)) */
static double refine_cum(double x, double V, double A, double w, const double *cs, int nc)
{
    double s = x + V;
    for (int i = 0; i < nc; ++i) s += A * w * 0.5 * sqrt(M_PI) * (erf((x - cs[i]) / w) - erf((-V - cs[i]) / w));
    return s;
}

/* the point where the normalised cumulative reaches u in [-1, 1]: bisection
 * on [-V, V] to the last representable midpoint (the cumulative is
 * increasing), ends exact */
static double refine_inverse(double u, double V, double A, double w, const double *cs, int nc)
{
    if (u <= -1.0) return -V;
    if (u >= 1.0) return V;
    const double t = 0.5 * (u + 1.0) * refine_cum(V, V, A, w, cs, nc);
    double lo = -V, hi = V;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (refine_cum(mid, V, A, w, cs, nc) < t)
            lo = mid;
        else
            hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* nodes, weights and dual cells [e0, e1] of one axis */
static void velocity_axis(int N, double lo, double hi, int rule, double beta, double *x, double *w, double *e0,
                          double *e1, double *d, double ramp, double rwidth, double rcentre, int jac)
{
    if (rule == OR_RULE_REFINED) {
        /* node i at u = (2i + 1 - N)/N, its dual cell between the images of
         * (2i - N)/N and (2i + 2 - N)/N; with the one bump at 0 the density
         * is even, and the negative half is the mirror of the positive one
         * so that nodes and faces are exactly antisymmetric */
        const double V = hi;
        double cs[2] = {0.0, rcentre};
        const int nc = rcentre != 0.0 ? 2 : 1;
        for (int m = 0; m <= 2 * N; ++m) {
            const int k = m - N; /* u = k / N */
            double v;
            if (nc == 1 && k == 0)
                v = 0.0; /* the centre of an even density */
            else if (nc == 1 && k < 0)
                v = -refine_inverse((double)(-k) / (double)N, V, ramp, rwidth, cs, nc);
            else
                v = refine_inverse((double)k / (double)N, V, ramp, rwidth, cs, nc);
            if (m % 2 == 0) {
                if (m / 2 < N) e0[m / 2] = v;
                if (m / 2 > 0) e1[m / 2 - 1] = v;
            } else {
                x[m / 2] = v;
            }
        }
        /* Jacobian weights: the normalised cumulative maps x(u) to u, so
         * x'(u) = total / (2 rho(x)) and the u-cell is 2/N wide */
        const double total = refine_cum(V, V, ramp, rwidth, cs, nc);
        for (int i = 0; i < N; ++i) {
            if (jac) {
                double rho = 1.0;
                for (int c = 0; c < nc; ++c) rho += ramp * exp(-((x[i] - cs[c]) / rwidth) * ((x[i] - cs[c]) / rwidth));
                w[i] = total / ((double)N * rho);
            } else {
                w[i] = e1[i] - e0[i];
            }
        }
        *d = 0.0;
        return;
    }
    if (rule == OR_RULE_STRETCHED) {
        /* node i at u = (2i + 1 - N)/N, its dual cell between the images of
         * u = (2i - N)/N and (2i + 2 - N)/N; the weight is the cell width */
        const double V = hi;
        for (int i = 0; i < N; ++i) {
            x[i] = stretch_map(V, beta, 2 * i + 1 - N, N);
            e0[i] = stretch_map(V, beta, 2 * i - N, N);
            e1[i] = stretch_map(V, beta, 2 * i + 2 - N, N);
            /* Jacobian weights: x'(u) = V beta cosh(beta u) / sinh(beta) */
            if (jac)
                w[i] = V * beta * cosh(beta * ((double)(2 * i + 1 - N) / (double)N)) / sinh(beta) * (2.0 / (double)N);
            else
                w[i] = e1[i] - e0[i];
        }
        *d = 0.0;
        return;
    }
    /* nodes c + (i - (N-1)/2) h about the box centre c: the same uniform
     * nodes as lo + i h (trapezoid) or lo + (i + 1/2) h (midpoint), written
     * so that a symmetric box gives exactly antisymmetric nodes; dual cells
     * x +- h/2 clipped to the box */
    double h = (rule == OR_RULE_TRAPEZOID) ? (hi - lo) / (double)(N - 1) : (hi - lo) / (double)N;
    double c = 0.5 * (lo + hi);
    for (int i = 0; i < N; ++i) {
        x[i] = c + ((double)i - 0.5 * (double)(N - 1)) * h;
        w[i] = (rule == OR_RULE_TRAPEZOID && (i == 0 || i == N - 1)) ? 0.5 * h : h;
        e0[i] = x[i] - 0.5 * h < lo ? lo : x[i] - 0.5 * h;
        e1[i] = x[i] + 0.5 * h > hi ? hi : x[i] + 0.5 * h;
    }
    *d = h;
}

/* dual cell of node i on one axis, clipped to the velocity box */
static void dual_edges(const or_state *s, int a, int i, double *e0, double *e1)
{
    *e0 = s->ed0[a][i];
    *e1 = s->ed1[a][i];
}

/* ------------------------------------------------------------------ */
/* cut-cell measures in velocity space (Section 3.2.3)                 */
/* ------------------------------------------------------------------ */

/* area of {v in [x0,x1]x[y0,y1] : nx*vx + ny*vy <= c} by clipping the
 * rectangle against the half-plane and applying the shoelace formula */
static double clip_area(double x0, double x1, double y0, double y1, double nx, double ny, double c)
{
    double px[4] = {x0, x1, x1, x0}, py[4] = {y0, y0, y1, y1};
    double qx[8], qy[8];
    int m = 0;
    for (int e = 0; e < 4; ++e) {
        int f = (e + 1) % 4;
        double dp = nx * px[e] + ny * py[e] - c;
        double dq = nx * px[f] + ny * py[f] - c;
        int ip = dp <= 0.0, iq = dq <= 0.0;
        if (ip) {
            qx[m] = px[e];
            qy[m] = py[e];
            ++m;
        }
        if (ip != iq) {
            double t = dp / (dp - dq);
            qx[m] = px[e] + t * (px[f] - px[e]);
            qy[m] = py[e] + t * (py[f] - py[e]);
            ++m;
        }
    }
    double A = 0.0;
    for (int e = 0; e < m; ++e) {
        int f = (e + 1) % m;
        A += qx[e] * qy[f] - qx[f] * qy[e];
    }
    return 0.5 * fabs(A);
}

static int cmp_d(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* volume of {v in box : n.v <= 0}: the cross-section area A(z) is piecewise
 * quadratic in z with breaks where the cutting line passes a corner of the
 * xy-rectangle; Simpson's rule is exact on each piece. */
static double clip_volume(const double e0[3], const double e1[3], const double n[3])
{
    if (n[2] == 0.0) return clip_area(e0[0], e1[0], e0[1], e1[1], n[0], n[1], 0.0) * (e1[2] - e0[2]);
    double zb[6];
    int m = 0;
    zb[m++] = e0[2];
    zb[m++] = e1[2];
    for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy) {
            double x = cx ? e1[0] : e0[0], y = cy ? e1[1] : e0[1];
            double z = -(n[0] * x + n[1] * y) / n[2];
            if (z > e0[2] && z < e1[2]) zb[m++] = z;
        }
    qsort(zb, m, sizeof(double), cmp_d);
    double V = 0.0;
    for (int p = 0; p + 1 < m; ++p) {
        double a = zb[p], b = zb[p + 1];
        if (b <= a) continue;
        double zm = 0.5 * (a + b);
        double fa = clip_area(e0[0], e1[0], e0[1], e1[1], n[0], n[1], -n[2] * a);
        double fm = clip_area(e0[0], e1[0], e0[1], e1[1], n[0], n[1], -n[2] * zm);
        double fb = clip_area(e0[0], e1[0], e0[1], e1[1], n[0], n[1], -n[2] * b);
        V += (b - a) / 6.0 * (fa + 4.0 * fm + fb);
    }
    return V;
}

/* classify every velocity node against the cut plane xi.n = 0 and compute
 * the incident-side measure (Section 3.2.3; snap rule R11) */
static void build_cut_sets(const or_state *s, const double n[3], unsigned char *cls, double *wg)
{
    int D = s->D;
    for (int k = 0; k < s->NV; ++k) {
        int id[3] = {k % s->c.vn[0], (k / s->c.vn[0]) % s->c.vn[1], D == 3 ? k / (s->c.vn[0] * s->c.vn[1]) : 0};
        double e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) dual_edges(s, a, id[a], &e0[a], &e1[a]);
        double dmin = INFINITY, dmax = -INFINITY, vmax = 0.0;
        for (int corner = 0; corner < (1 << D); ++corner) {
            double v[3];
            for (int a = 0; a < D; ++a) v[a] = (corner >> a & 1) ? e1[a] : e0[a];
            double d = 0.0, r = 0.0;
            for (int a = 0; a < D; ++a) {
                d += v[a] * n[a];
                r += v[a] * v[a];
            }
            r = sqrt(r);
            if (d < dmin) dmin = d;
            if (d > dmax) dmax = d;
            if (r > vmax) vmax = r;
        }
        double eps = 1e-12 * vmax;
        double dn = 0.0;
        for (int a = 0; a < D; ++a) dn += s->xi[3 * k + a] * n[a];
        int cut = (dmin < -eps) && (dmax > eps);
        if ((s->c.flags & OR_FLAG_NO_CUTCELL) || !cut) {
            cls[k] = dn <= 0.0 ? CL_GAS : CL_SOLID;
            wg[k] = dn <= 0.0 ? s->w[k] : 0.0;
        } else {
            cls[k] = dn <= 0.0 ? CL_CUT_G : CL_CUT_S;
            if (D == 2)
                wg[k] = clip_area(e0[0], e1[0], e0[1], e1[1], n[0], n[1], 0.0);
            else
                wg[k] = clip_volume(e0, e1, n);
            if (s->c.vweights == OR_WEIGHTS_JACOBIAN) {
                /* the incident fraction of the dual cell, of the node's weight */
                double vol = 1.0;
                for (int a = 0; a < D; ++a) vol *= e1[a] - e0[a];
                wg[k] = wg[k] / vol * s->w[k];
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* kinetic model (Section 2.1; reduced forms of Section 4)            */
/* ------------------------------------------------------------------ */

/* moments of one cell: rho, U, T, q (moment equations of Section 2.1 with
 * p = rho T / 2 in the units of Section 4) */
static void cell_moments(const or_state *s, const double *f0, const double *f1, double out[8])
{
    int D = s->D;
    double rho = 0.0, m[3] = {0, 0, 0}, E2 = 0.0;
    for (int k = 0; k < s->NV; ++k) {
        const double *x = &s->xi[3 * k];
        double x2 = 0.0;
        for (int a = 0; a < D; ++a) x2 += x[a] * x[a];
        rho += s->w[k] * f0[k];
        for (int a = 0; a < D; ++a) m[a] += s->w[k] * x[a] * f0[k];
        if (D == 2)
            E2 += s->w[k] * (x2 * f0[k] + f1[k]);
        else
            E2 += s->w[k] * x2 * f0[k];
    }
    double U[3] = {0, 0, 0}, U2 = 0.0;
    for (int a = 0; a < D; ++a) {
        U[a] = m[a] / rho;
        U2 += U[a] * U[a];
    }
    double rhoE = 0.5 * E2;
    double T = 4.0 * (rhoE - 0.5 * rho * U2) / (3.0 * rho);
    double q[3] = {0, 0, 0};
    for (int k = 0; k < s->NV; ++k) {
        const double *x = &s->xi[3 * k];
        double cc[3] = {0, 0, 0}, c2 = 0.0;
        for (int a = 0; a < D; ++a) {
            cc[a] = x[a] - U[a];
            c2 += cc[a] * cc[a];
        }
        for (int a = 0; a < D; ++a) {
            if (D == 2)
                q[a] += s->w[k] * cc[a] * (c2 * f0[k] + f1[k]);
            else
                q[a] += s->w[k] * cc[a] * c2 * f0[k];
        }
    }
    out[0] = rho;
    for (int a = 0; a < 3; ++a) out[1 + a] = U[a];
    out[4] = T;
    for (int a = 0; a < 3; ++a) out[5 + a] = 0.5 * q[a];
}

/* relaxation time tau = mu / p with mu = mu0 T^omega (VHS law of Section 4) */
static double relax_time(const or_state *s, double rho, double T)
{
    double mu = s->mu0 * pow(T, s->c.omega);
    double p = 0.5 * rho * T;
    return mu / p;
}

/* Shakhov equilibrium: reduced H^S, B^S (2D) or g^S (3D), Section 4 / 2.1 */
static void shakhov(const or_state *s, const double mom[8], double *g0, double *g1)
{
    int D = s->D;
    double rho = mom[0], T = mom[4];
    const double *U = &mom[1], *q = &mom[5];
    double coef = 4.0 * (1.0 - s->c.Pr) / (5.0 * rho * T * T);
    double pref = (D == 2) ? rho / (M_PI * T) : rho / pow(M_PI * T, 1.5);
    for (int k = 0; k < s->NV; ++k) {
        const double *x = &s->xi[3 * k];
        double c2 = 0.0, cq = 0.0;
        for (int a = 0; a < D; ++a) {
            double cc = x[a] - U[a];
            c2 += cc * cc;
            cq += cc * q[a];
        }
        double H = pref * exp(-c2 / T);
        if (D == 2) {
            double B = 0.5 * T * H;
            g0[k] = H * (1.0 + coef * cq * (2.0 * c2 / T - 4.0));
            g1[k] = B * (1.0 + coef * cq * (2.0 * c2 / T - 2.0));
        } else {
            g0[k] = H * (1.0 + coef * cq * (2.0 * c2 / T - 5.0));
        }
    }
}

/* plain Maxwellian (H, B) or g with given rho, U, T */
static void maxwellian(const or_state *s, double rho, const double U[3], double T, double *g0, double *g1)
{
    int D = s->D;
    double pref = (D == 2) ? rho / (M_PI * T) : rho / pow(M_PI * T, 1.5);
    for (int k = 0; k < s->NV; ++k) {
        double c2 = 0.0;
        for (int a = 0; a < D; ++a) {
            double cc = s->xi[3 * k + a] - U[a];
            c2 += cc * cc;
        }
        g0[k] = pref * exp(-c2 / T);
        if (g1) g1[k] = 0.5 * T * g0[k];
    }
}

/* ------------------------------------------------------------------ */
/* construction                                                        */
/* ------------------------------------------------------------------ */

static double seg_root(const or_state *s, const double xg[3], const double xd[3], int a)
{
    const or_case *c = &s->c;
    if (c->gkind == OR_G_CIRCLE || c->gkind == OR_G_SPHERE) {
        /* crossing of the axis line with the circle / sphere in closed form:
         * (t - c_a)^2 = R^2 - sum_{b != a} (x_b - c_b)^2, on the donor side.
         * Bisection on phi cannot place a grazing crossing better than about
         * sqrt(ulp(R^2)) because x^2 + rest rounds to rest there. */
        double rest = 0.0;
        for (int b = 0; b < s->D; ++b)
            if (b != a) rest += (xg[b] - c->gcen[b]) * (xg[b] - c->gcen[b]);
        double h = c->gsize[0] * c->gsize[0] - rest;
        double sgn = xd[a] > xg[a] ? 1.0 : -1.0;
        double t = c->gcen[a] + sgn * sqrt(h > 0.0 ? h : 0.0);
        double lo = xg[a] < xd[a] ? xg[a] : xd[a], hi = xg[a] < xd[a] ? xd[a] : xg[a];
        return t < lo ? lo : (t > hi ? hi : t);
    }
    /* other shapes: bisection on phi along the axis segment from the ghost
     * centre (phi<0) to the donor centre (phi>=0) */
    double lo = xg[a], hi = xd[a];
    double x[3] = {xg[0], xg[1], xg[2]};
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        x[a] = mid;
        if (phi(s, x) < 0.0)
            lo = mid;
        else
            hi = mid;
    }
    return hi;
}

void or_destroy(void *h);

void *or_create(const or_case *cs, int *err)
{
    *err = 0;
    or_state *s = (or_state *)calloc(1, sizeof(or_state));
    s->c = *cs;
    int D = s->D = cs->dim;
    s->NA = (D == 2) ? 2 : 1;
    s->Nc = 1;
    s->NV = 1;
    for (int a = 0; a < D; ++a) {
        s->Nc *= cs->n[a];
        s->NV *= cs->vn[a];
        s->dx[a] = (cs->hi[a] - cs->lo[a]) / (double)cs->n[a];
    }
    if (D == 2) {
        s->c.n[2] = 1;
        s->c.vn[2] = 1;
    }
    if (cs->vrule == OR_RULE_STRETCHED)
        for (int a = 0; a < D; ++a)
            if (!(cs->vstretch > 0.0) || cs->vlo[a] != -cs->vhi[a]) *err = 1;
    if (cs->vrule == OR_RULE_REFINED)
        for (int a = 0; a < D; ++a)
            if (!(cs->vref_amp >= 0.0) || !(cs->vref_width > 0.0) || cs->vlo[a] != -cs->vhi[a] ||
                !(fabs(cs->vref_centre[a]) < cs->vhi[a]))
                *err = 1;
    if (cs->vweights != OR_WEIGHTS_CELL &&
        !(cs->vweights == OR_WEIGHTS_JACOBIAN && (cs->vrule == OR_RULE_STRETCHED || cs->vrule == OR_RULE_REFINED)))
        *err = 1;
    if (cs->vrule == OR_RULE_REFINED && cs->outer == OR_SPECULAR)
        for (int a = 0; a < D; ++a)
            if (cs->vref_centre[a] != 0.0) *err = 1; /* mirrored nodes must be nodes */
    /* velocity grid */
    for (int a = 0; a < D; ++a) {
        s->xi1[a] = (double *)malloc(sizeof(double) * cs->vn[a]);
        s->w1[a] = (double *)malloc(sizeof(double) * cs->vn[a]);
        s->ed0[a] = (double *)malloc(sizeof(double) * cs->vn[a]);
        s->ed1[a] = (double *)malloc(sizeof(double) * cs->vn[a]);
        velocity_axis(cs->vn[a], cs->vlo[a], cs->vhi[a], cs->vrule, cs->vstretch, s->xi1[a], s->w1[a], s->ed0[a],
                      s->ed1[a], &s->dxi[a], cs->vref_amp, cs->vref_width, cs->vref_centre[a],
                      cs->vweights == OR_WEIGHTS_JACOBIAN);
        s->maxabs[a] = 0.0;
        for (int i = 0; i < cs->vn[a]; ++i)
            if (fabs(s->xi1[a][i]) > s->maxabs[a]) s->maxabs[a] = fabs(s->xi1[a][i]);
    }
    s->xi = (double *)calloc((size_t)3 * s->NV, sizeof(double));
    s->w = (double *)malloc(sizeof(double) * s->NV);
    for (int k = 0; k < s->NV; ++k) {
        int id[3] = {k % s->c.vn[0], (k / s->c.vn[0]) % s->c.vn[1], D == 3 ? k / (s->c.vn[0] * s->c.vn[1]) : 0};
        double w = 1.0;
        for (int a = 0; a < D; ++a) {
            s->xi[3 * k + a] = s->xi1[a][id[a]];
            w *= s->w1[a][id[a]];
        }
        s->w[k] = w;
    }
    /* viscosity coefficient (Section 4, VHS reference viscosity) */
    double al = cs->avhs, om = cs->omega;
    s->mu0 = 5.0 * (al + 1.0) * (al + 2.0) * sqrt(M_PI) / (4.0 * al * (5.0 - 2.0 * om) * (7.0 - 2.0 * om)) * cs->Kn;
    s->Uinf = cs->Ma * sqrt(cs->gam / 2.0);

    /* classification (Section 3.2.1): solid iff phi(centre) < 0 */
    s->solid = (unsigned char *)calloc(s->Nc, 1);
    for (int c = 0; c < s->Nc; ++c) {
        int ijk[3];
        cell_ijk(s, c, ijk);
        double x[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) x[a] = xc(s, a, ijk[a]);
        s->solid[c] = (cs->gkind != OR_G_NONE) && phi(s, x) < 0.0;
        if (s->solid[c])
            for (int a = 0; a < D; ++a)
                if (ijk[a] < 3 || ijk[a] > cs->n[a] - 4) *err = 2;
    }
    if ((cs->outer == OR_WALLS || cs->outer == OR_SPECULAR) && D != 2) *err = 1;
    if (cs->outer == OR_SPECULAR)
        for (int a = 0; a < D; ++a)
            if (cs->vlo[a] != -cs->vhi[a]) *err = 1; /* mirrored nodes must be nodes */
    if (*err) {
        or_destroy(s);
        return NULL;
    }
    if (cs->outer == OR_WALLS || cs->outer == OR_SPECULAR)
        for (int A = 0; A < s->NA; ++A)
            s->wgh[A] = (double *)calloc((size_t)2 * (cs->n[0] + cs->n[1]) * s->NV, sizeof(double));
    /* pairs: one per (ghost, fluid face neighbour), ordered by ghost index,
     * then axis, then side (-1 before +1) */
    s->pnb = (int *)malloc(sizeof(int) * 6 * s->Nc);
    for (int i = 0; i < 6 * s->Nc; ++i) s->pnb[i] = -1;
    int cap = 16;
    s->pairs = (or_pair *)calloc(cap, sizeof(or_pair));
    s->npairs = 0;
    s->nghost = 0;
    for (int c = 0; c < s->Nc; ++c) {
        if (!s->solid[c]) continue;
        int ijk[3];
        cell_ijk(s, c, ijk);
        int isghost = 0;
        for (int a = 0; a < D; ++a)
            for (int sg = -1; sg <= 1; sg += 2) {
                int nb[3] = {ijk[0], ijk[1], ijk[2]};
                nb[a] += sg;
                int d = cell_id(s, nb);
                if (s->solid[d]) continue;
                isghost = 1;
                if (s->npairs == cap) {
                    cap *= 2;
                    s->pairs = (or_pair *)realloc(s->pairs, cap * sizeof(or_pair));
                }
                or_pair *p = &s->pairs[s->npairs];
                memset(p, 0, sizeof(*p));
                p->gc = c;
                p->dc = d;
                p->axis = a;
                p->sign = sg;
                double xg[3] = {0, 0, 0}, xd[3] = {0, 0, 0};
                for (int b = 0; b < D; ++b) {
                    xg[b] = xc(s, b, ijk[b]);
                    xd[b] = xc(s, b, nb[b]);
                }
                /* intersect point (Section 3.2.1) */
                for (int b = 0; b < 3; ++b) p->xw[b] = xg[b];
                p->xw[a] = seg_root(s, xg, xd, a);
                normal(s, p->xw, p->nw);
                {
                    double r[3] = {0, 0, 0};
                    for (int b = 0; b < D; ++b) r[b] = p->xw[b] - cs->gcen[b];
                    const double *O = cs->Ow;
                    double ox[3] = {O[1] * r[2] - O[2] * r[1], O[2] * r[0] - O[0] * r[2], O[0] * r[1] - O[1] * r[0]};
                    for (int b = 0; b < 3; ++b) p->uw[b] = b < D ? cs->Uw[b] + ox[b] : 0.0;
                }
                /* shifted point y_sp = y_w + (y_dc - y_gc)/2 (shifted-point equation) */
                for (int b = 0; b < 3; ++b) p->xsp[b] = p->xw[b];
                p->xsp[a] = p->xw[a] + (xd[a] - xg[a]) / 2.0;
                /* auxiliary cell next to the donor along the same axis */
                int an[3] = {nb[0], nb[1], nb[2]};
                an[a] += sg;
                p->ac = (in_grid(s, an) && !s->solid[cell_id(s, an)] && !(cs->flags & OR_FLAG_NO_AUX)) ? cell_id(s, an)
                                                                                                   : -1;
                /* surface cells: fluid cells of the Moore neighbourhood */
                p->ns = 0;
                for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dxo = -1; dxo <= 1; ++dxo) {
                            if (dxo == 0 && dy == 0 && dz == 0) continue;
                            int m[3] = {ijk[0] + dxo, ijk[1] + dy, ijk[2] + dz};
                            if (!in_grid(s, m)) continue;
                            int mc = cell_id(s, m);
                            if (s->solid[mc]) continue;
                            p->sc[p->ns] = mc;
                            double rr = 0.0;
                            for (int b = 0; b < D; ++b) {
                                p->r[p->ns][b] = xc(s, b, m[b]) - xg[b];
                                rr += p->r[p->ns][b] * p->r[p->ns][b];
                            }
                            rr = sqrt(rr);
                            for (int b = 0; b < D; ++b) p->rh[p->ns][b] = p->r[p->ns][b] / rr;
                            p->ns++;
                        }
                p->cls = (unsigned char *)malloc(s->NV);
                p->wg = (double *)malloc(sizeof(double) * s->NV);
                build_cut_sets(s, p->nw, p->cls, p->wg);
                /* the donor sees this pair when looking toward the ghost */
                int side = -sg;
                s->pnb[6 * d + 2 * a + (side > 0)] = s->npairs;
                s->npairs++;
            }
        s->nghost += isghost;
    }
    size_t nf = (size_t)s->Nc * s->NV;
    for (int A = 0; A < s->NA; ++A) {
        s->f[A] = (double *)calloc(nf, sizeof(double));
        s->fn[A] = (double *)calloc(nf, sizeof(double));
        s->fs[A] = (double *)malloc(sizeof(double) * s->NV);
        size_t np = (size_t)(s->npairs > 0 ? s->npairs : 1) * s->NV;
        s->fsp[A] = (double *)calloc(np, sizeof(double));
        s->fgc[A] = (double *)calloc(np, sizeof(double));
        s->fiw[A] = (double *)calloc(np, sizeof(double));
        s->fss[A] = (double *)calloc(np, sizeof(double));
        s->fw[A] = (double *)calloc(np, sizeof(double));
        s->gh[A] = (double *)calloc(np, sizeof(double));
        s->fc[A] = (double *)calloc(np, sizeof(double));
    }
    s->rhow = (double *)calloc(s->npairs > 0 ? s->npairs : 1, sizeof(double));
    s->mom = (double *)calloc((size_t)8 * s->Nc, sizeof(double));
    s->tau = (double *)calloc(s->Nc, sizeof(double));
    double Uf[3] = {s->Uinf, 0, 0};
    maxwellian(s, 1.0, Uf, 1.0, s->fs[0], s->NA == 2 ? s->fs[1] : NULL);
    return s;
}

void or_destroy(void *h)
{
    or_state *s = (or_state *)h;
    if (!s) return;
    for (int a = 0; a < 3; ++a) {
        free(s->xi1[a]);
        free(s->w1[a]);
        free(s->ed0[a]);
        free(s->ed1[a]);
    }
    free(s->xi);
    free(s->w);
    free(s->solid);
    free(s->pnb);
    for (int p = 0; p < s->npairs; ++p) {
        free(s->pairs[p].cls);
        free(s->pairs[p].wg);
    }
    free(s->pairs);
    for (int A = 0; A < 2; ++A) {
        free(s->f[A]);
        free(s->fn[A]);
        free(s->fs[A]);
        free(s->fsp[A]);
        free(s->fgc[A]);
        free(s->fiw[A]);
        free(s->fss[A]);
        free(s->fw[A]);
        free(s->gh[A]);
        free(s->fc[A]);
    }
    free(s->rhow);
    free(s->wgh[0]);
    free(s->wgh[1]);
    free(s->mom);
    free(s->tau);
    free(s);
}

/* ------------------------------------------------------------------ */
/* state access                                                        */
/* ------------------------------------------------------------------ */

/* freestream Maxwellian times (1 + amp*u), u given per (cell, node) */
void or_init_freestream(void *h, const double *u0, const double *u1, double amp)
{
    or_state *s = (or_state *)h;
    const double *u[2] = {u0, u1};
    for (int A = 0; A < s->NA; ++A)
        for (int c = 0; c < s->Nc; ++c)
            for (int k = 0; k < s->NV; ++k) {
                size_t i = (size_t)c * s->NV + k;
                s->f[A][i] = s->fs[A][k] * (1.0 + (u[A] ? amp * u[A][i] : 0.0));
            }
    s->step = 0;
    s->time = 0.0;
}

void or_set_state(void *h, const double *f0, const double *f1)
{
    or_state *s = (or_state *)h;
    size_t nf = (size_t)s->Nc * s->NV;
    memcpy(s->f[0], f0, nf * sizeof(double));
    if (s->NA == 2) memcpy(s->f[1], f1, nf * sizeof(double));
}

void or_get_state(void *h, double *f0, double *f1)
{
    or_state *s = (or_state *)h;
    size_t nf = (size_t)s->Nc * s->NV;
    memcpy(f0, s->f[0], nf * sizeof(double));
    if (s->NA == 2 && f1) memcpy(f1, s->f[1], nf * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* one time step                                                       */
/* ------------------------------------------------------------------ */

static void all_moments(or_state *s)
{
#pragma omp parallel for schedule(static)
    for (int c = 0; c < s->Nc; ++c) {
        if (s->solid[c]) {
            for (int i = 0; i < 8; ++i) s->mom[8 * c + i] = NAN;
            s->tau[c] = NAN;
            continue;
        }
        const double *f0 = s->f[0] + (size_t)c * s->NV;
        const double *f1 = s->NA == 2 ? s->f[1] + (size_t)c * s->NV : NULL;
        cell_moments(s, f0, f1, &s->mom[8 * c]);
        s->tau[c] = relax_time(s, s->mom[8 * c], s->mom[8 * c + 4]);
    }
}

/* time step (reading R14): positivity bound of first-order upwinding plus
 * explicit relaxation, with the smallest relaxation time of the state; the
 * implicit relaxation (R30) leaves only the upwinding bound */
static double time_step(const or_state *s)
{
    double tmin = INFINITY;
    for (int c = 0; c < s->Nc; ++c)
        if (!s->solid[c] && s->tau[c] < tmin) tmin = s->tau[c];
    double adv = 0.0;
    for (int a = 0; a < s->D; ++a) adv += s->maxabs[a] / s->dx[a];
    if (s->c.flags & OR_FLAG_IMPLICIT) return s->c.cfl / adv;
    return s->c.cfl / (adv + 1.0 / tmin);
}

/* fluid-only slope of a surface cell along axis b (reading R9) */
static double fluid_slope(const or_state *s, const double *f, int j, int b, int k)
{
    int ijk[3];
    cell_ijk(s, j, ijk);
    int L[3] = {ijk[0], ijk[1], ijk[2]}, R[3] = {ijk[0], ijk[1], ijk[2]};
    L[b] -= 1;
    R[b] += 1;
    int lf = in_grid(s, L) && !s->solid[cell_id(s, L)];
    int rf = in_grid(s, R) && !s->solid[cell_id(s, R)];
    double fj = f[(size_t)j * s->NV + k];
    double h = s->dx[b];
    if (lf && rf) {
        double fl = f[(size_t)cell_id(s, L) * s->NV + k], fr = f[(size_t)cell_id(s, R) * s->NV + k];
        return vanleer((fj - fl) / h, (fr - fj) / h);
    }
    if (rf) return (f[(size_t)cell_id(s, R) * s->NV + k] - fj) / h;
    if (lf) return (fj - f[(size_t)cell_id(s, L) * s->NV + k]) / h;
    return 0.0;
}

/* multilinear interpolation of an array on the velocity nodes; zero outside
 * the node hull (reading R12) */
static double vel_interp(const or_state *s, const double *g, const double v[3])
{
    int D = s->D;
    int i0[3] = {0, 0, 0};
    double t[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
        int N = s->c.vn[a];
        const double *x = s->xi1[a];
        if (v[a] < x[0] || v[a] > x[N - 1]) return 0.0;
        int i = 0;
        while (i < N - 2 && v[a] > x[i + 1]) ++i;
        i0[a] = i;
        t[a] = (v[a] - x[i]) / (x[i + 1] - x[i]);
    }
    double acc = 0.0;
    for (int corner = 0; corner < (1 << D); ++corner) {
        double wgt = 1.0;
        int id[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            int up = corner >> a & 1;
            id[a] = i0[a] + up;
            wgt *= up ? t[a] : 1.0 - t[a];
        }
        int k = id[0] + s->c.vn[0] * (id[1] + s->c.vn[1] * id[2]);
        acc += wgt * g[k];
    }
    return acc;
}

/* wall density and wall distribution at one wall point with normal n and
 * wall velocity uw, from the incident distribution fi and its mirrored part
 * fs (arrays offset by o): zero net normal mass flux with cut-cell weights
 * (cut-cell no-penetration equation; readings R2, R3), Maxwell reflection
 * with accommodation alpha and the wall Maxwellian at (uw, T_w) (Section
 * 2.3), general wall condition and cut-cell blend */
static void wall_distribution(const or_state *s, const double n[3], const double uw[3], const unsigned char *cls,
                              const double *wg, double *const fi[2], double *const fs[2], size_t o, double *rhow,
                              double *const fw[2])
{
    int D = s->D, NV = s->NV;
    double Tw = s->c.Tw, al = s->c.alpha;
    double hw_pref = (D == 2) ? 1.0 / (M_PI * Tw) : 1.0 / pow(M_PI * Tw, 1.5);
    double num = 0.0, den = 0.0;
    for (int k = 0; k < NV; ++k) {
        const double *x = &s->xi[3 * k];
        double dn = 0.0, x2 = 0.0;
        for (int b = 0; b < D; ++b) {
            dn += x[b] * n[b];
            x2 += (x[b] - uw[b]) * (x[b] - uw[b]);
        }
        double Hw = hw_pref * exp(-x2 / Tw);
        if (cls[k] == CL_GAS) {
            num += s->w[k] * dn * fi[0][o + k];
        } else if (cls[k] == CL_SOLID) {
            num += (1.0 - al) * s->w[k] * dn * fs[0][o + k];
            den += s->w[k] * dn * Hw;
        } else {
            num += wg[k] * dn * fi[0][o + k];
            num += (1.0 - al) * (s->w[k] - wg[k]) * dn * fs[0][o + k];
            den += (s->w[k] - wg[k]) * dn * Hw;
        }
    }
    double rw = (al > 0.0) ? -num / (al * den) : 0.0;
    *rhow = rw;
    for (int A = 0; A < s->NA; ++A)
        for (int k = 0; k < NV; ++k) {
            double x2 = 0.0;
            for (int b = 0; b < D; ++b) x2 += (s->xi[3 * k + b] - uw[b]) * (s->xi[3 * k + b] - uw[b]);
            double Hw = hw_pref * exp(-x2 / Tw);
            if (A == 1) Hw *= 0.5 * Tw;
            double f_i = fi[A][o + k];
            double f_r = al * rw * Hw + (1.0 - al) * fs[A][o + k];
            if (cls[k] == CL_GAS)
                fw[A][o + k] = f_i;
            else if (cls[k] == CL_SOLID)
                fw[A][o + k] = f_r;
            else
                fw[A][o + k] = (wg[k] * f_i + (s->w[k] - wg[k]) * f_r) / s->w[k];
        }
}

/* specular part: the incident array interpolated at the mirrored velocity
 * xi - 2 (xi.n) n (reading R12) */
static void specular_part(const or_state *s, const double n[3], const double *fi, double *fs)
{
    int D = s->D;
    for (int k = 0; k < s->NV; ++k) {
        const double *x = &s->xi[3 * k];
        double dn = 0.0;
        for (int b = 0; b < D; ++b) dn += x[b] * n[b];
        double v[3] = {0, 0, 0};
        for (int b = 0; b < D; ++b) v[b] = x[b] - 2.0 * dn * n[b];
        fs[k] = vel_interp(s, fi, v);
    }
}

/* xi . r_hat for the upwind weights, with |xi . r_hat| <= 1e-12 |xi| taken
 * as exactly zero (reading R25): the weight rule switches to 1/N_S when the
 * sum of squared positive parts vanishes, and without the snap that switch
 * would be decided by round-off for velocities orthogonal to r_hat */
static double upwind_dot(const or_state *s, const double *x, const double *rh)
{
    double d = 0.0, x2 = 0.0;
    for (int b = 0; b < s->D; ++b) {
        d += x[b] * rh[b];
        x2 += x[b] * x[b];
    }
    return (fabs(d) <= 1e-12 * sqrt(x2)) ? 0.0 : d;
}

/* upwind interpolation weights of the ns surface cells of pair p at node
 * velocity x (Section 3.2.2, sign by reading R4): the squared positive part
 * of -xi . r_hat_j, normalised; 1/N_S when every part is zero */
static void upwind_weights(const or_state *s, const or_pair *p, const double *x, double *w)
{
    double m2[26], sum = 0.0;
    for (int j = 0; j < p->ns; ++j) {
        double d = upwind_dot(s, x, p->rh[j]);
        double m = -d > 0.0 ? -d : 0.0;
        m2[j] = m * m;
        sum += m2[j];
    }
    for (int j = 0; j < p->ns; ++j) w[j] = (sum != 0.0) ? m2[j] / sum : 1.0 / p->ns;
}

/* ghost-cell construction for every pair (Section 3.2.1 steps 1-4 with the
 * weights of 3.2.2 and the velocity-space cut-cell correction of 3.2.3) */
static void ib_fill(or_state *s)
{
    int D = s->D, NV = s->NV;
    double al = s->c.alpha;
#pragma omp parallel for schedule(dynamic)
    for (int ip = 0; ip < s->npairs; ++ip) {
        const or_pair *p = &s->pairs[ip];
        int a = p->axis;
        size_t o = (size_t)ip * NV;
        int gij[3], dij[3];
        cell_ijk(s, p->gc, gij);
        cell_ijk(s, p->dc, dij);
        double ygc = xc(s, a, gij[a]), ydc = xc(s, a, dij[a]);
        double yw = p->xw[a], ysp = p->xsp[a];
        for (int A = 0; A < s->NA; ++A) {
            const double *f = s->f[A];
            for (int k = 0; k < NV; ++k) {
                const double *x = &s->xi[3 * k];
                /* 1. shifted point from the donor with the auxiliary slope */
                double fdc = f[(size_t)p->dc * NV + k];
                double sdc = 0.0;
                if (p->ac >= 0) {
                    int aij[3];
                    cell_ijk(s, p->ac, aij);
                    sdc = (f[(size_t)p->ac * NV + k] - fdc) / (xc(s, a, aij[a]) - ydc);
                }
                double fsp = fdc + sdc * (ysp - ydc);
                double fgc = 0.0;
                if (s->c.flags & OR_FLAG_NAIVE) {
                    /* 2'. naive linear extrapolation of donor and auxiliary
                     * cell along the axis (Section 3.3.3 ablation) */
                    fgc = fdc + sdc * (ygc - ydc);
                } else {
                /* 2. upwind-weighted ghost interpolation (reading R4 for the sign) */
                double wu[26];
                upwind_weights(s, p, x, wu);
                for (int j = 0; j < p->ns; ++j) {
                    const double wj = (s->c.flags & OR_FLAG_NO_UPWIND) ? 1.0 / p->ns : wu[j];
                    double sr = 0.0;
                    for (int b = 0; b < D; ++b) sr += fluid_slope(s, f, p->sc[j], b, k) * p->r[j][b];
                    fgc += wj * (f[(size_t)p->sc[j] * NV + k] - sr);
                }
                }
                /* 3. incident distribution at the intersect point */
                double fiw = fsp + (fgc - fsp) / (ygc - ysp) * (yw - ysp);
                if (fiw < 0.0) fiw = 0.0; /* distributions are non-negative (reading R28) */
                s->fsp[A][o + k] = fsp;
                s->fgc[A][o + k] = fgc;
                s->fiw[A][o + k] = fiw;
            }
            /* specular part at the mirrored velocity (reading R12) */
            if (al < 1.0)
                specular_part(s, p->nw, s->fiw[A] + o, s->fss[A] + o);
            else
                for (int k = 0; k < NV; ++k) s->fss[A][o + k] = 0.0;
        }
        double yface = ygc + 0.5 * p->sign * s->dx[a];
        wall_distribution(s, p->nw, p->uw, p->cls, p->wg, s->fiw, s->fss, o, &s->rhow[ip], s->fw);
        for (int A = 0; A < s->NA; ++A)
            for (int k = 0; k < NV; ++k) {
                double fsp = s->fsp[A][o + k], fw = s->fw[A][o + k];
                double sig = (fw - fsp) / (yw - ysp); /* ghost-side slope (reading R8) */
                double gval = fsp + sig * (ygc - ysp);
                /* reading R28: the ghost value and the face value stay
                 * non-negative; with the face limit option the face value,
                 * taken on the same line, goes no further than the wall
                 * value when the face lies beyond the wall */
                double t = (yface - ysp) / (yw - ysp);
                if ((s->c.flags & OR_FLAG_FACE_LIMIT) && t > 1.0) t = 1.0;
                double fval = fsp + (fw - fsp) * t;
                s->gh[A][o + k] = gval < 0.0 ? 0.0 : gval;
                s->fc[A][o + k] = fval < 0.0 ? 0.0 : fval;
            }
    }
}

/* OR_WALLS, OR_SPECULAR: ghost row of boundary cell (i, j) for the wall on
 * side `side` of axis a */
static size_t wall_row(const or_state *s, int a, int side, const int ijk[3])
{
    const int nx = s->c.n[0], ny = s->c.n[1];
    if (a == 0) return (size_t)(side < 0 ? 0 : ny) + ijk[1];
    return (size_t)(2 * ny + (side < 0 ? 0 : nx)) + ijk[0];
}

/* Diffuse outer walls (reading R29: the wall model of Section 2.3 applied at
 * the domain faces).  For each boundary cell and wall, the ghost layer holds
 * the wall Maxwellian at (U_wall, T_w) with the density rho_w that makes the
 * net normal mass flux through the wall face zero for the first-order
 * outgoing face values f of the boundary cell, on the velocities leaving the
 * wall, and the cell's own value f on the velocities toward the wall (zero
 * gradient); both ghost layers are equal and their slope is zero. */
static void wall_fill(or_state *s)
{
    const int NV = s->NV;
    double *hw = (double *)malloc(sizeof(double) * NV), *bw = (double *)malloc(sizeof(double) * NV);
    for (int a = 0; a < 2; ++a)
        for (int sd = -1; sd <= 1; sd += 2) {
            double U[3] = {(a == 1 && sd > 0) ? s->c.lid_u : 0.0, 0.0, 0.0};
            maxwellian(s, 1.0, U, s->c.Tw, hw, bw);
            const int nb = s->c.n[1 - a];
            for (int b = 0; b < nb; ++b) {
                int ijk[3] = {0, 0, 0};
                ijk[a] = sd < 0 ? 0 : s->c.n[a] - 1;
                ijk[1 - a] = b;
                const size_t o = (size_t)cell_id(s, ijk) * NV;
                double out = 0.0, in = 0.0;
                for (int k = 0; k < NV; ++k) {
                    const double xn = sd * s->xi[3 * k + a]; /* > 0: toward the wall */
                    if (xn > 0.0)
                        out += s->w[k] * xn * s->f[0][o + k];
                    else if (xn < 0.0)
                        in -= s->w[k] * xn * hw[k];
                }
                const double rw = out / in;
                const size_t r = wall_row(s, a, sd, ijk) * NV;
                for (int k = 0; k < NV; ++k) {
                    const double xn = sd * s->xi[3 * k + a];
                    s->wgh[0][r + k] = xn < 0.0 ? rw * hw[k] : s->f[0][o + k];
                    s->wgh[1][r + k] = xn < 0.0 ? rw * bw[k] : s->f[1][o + k];
                }
            }
        }
    free(hw);
    free(bw);
}

/* Specular outer walls (reading R32: the wall model of Section 2.3 with
 * alpha = 0 at the domain faces, in the form of reading R29).  For each
 * boundary cell and wall, the ghost layer holds on the velocities leaving
 * the wall the cell's own value at the mirrored velocity (the velocity with
 * its normal component reversed, a node of the symmetric velocity grid),
 * and on the others the cell's own value; both ghost layers are equal.  The
 * face values of a velocity and of its mirror are then the same cell value,
 * so the walls pass no mass and no energy. */
static void specular_fill(or_state *s)
{
    const int NV = s->NV;
    for (int a = 0; a < 2; ++a)
        for (int sd = -1; sd <= 1; sd += 2) {
            const int nb = s->c.n[1 - a];
            for (int b = 0; b < nb; ++b) {
                int ijk[3] = {0, 0, 0};
                ijk[a] = sd < 0 ? 0 : s->c.n[a] - 1;
                ijk[1 - a] = b;
                const size_t o = (size_t)cell_id(s, ijk) * NV;
                const size_t r = wall_row(s, a, sd, ijk) * NV;
                for (int k = 0; k < NV; ++k) {
                    const double xn = sd * s->xi[3 * k + a]; /* > 0: toward the wall */
                    int id[2] = {k % s->c.vn[0], k / s->c.vn[0]};
                    id[a] = s->c.vn[a] - 1 - id[a];
                    const int km = xn < 0.0 ? id[0] + s->c.vn[0] * id[1] : k;
                    s->wgh[0][r + k] = s->f[0][o + km];
                    s->wgh[1][r + k] = s->f[1][o + km];
                }
            }
        }
}

/* value seen by fluid cell c at c + side*e_a; kind: 0 fluid, 1 outer
 * freestream or wall ghost, 2 immersed-boundary ghost.  *nbc returns the fluid
 * neighbour index (after periodic wrap) or -1. */
static double nb_value(const or_state *s, int A, int c, int a, int side, int k, int *kind, int *nbc)
{
    int ijk[3];
    cell_ijk(s, c, ijk);
    ijk[a] += side;
    if (ijk[a] < 0 || ijk[a] >= s->c.n[a]) {
        if (s->c.outer == OR_FREESTREAM) {
            *kind = 1;
            *nbc = -1;
            return s->fs[A][k];
        }
        if (s->c.outer == OR_WALLS || s->c.outer == OR_SPECULAR) {
            int bc[3];
            cell_ijk(s, c, bc);
            *kind = 1;
            *nbc = -1;
            return s->wgh[A][wall_row(s, a, side, bc) * s->NV + k];
        }
        ijk[a] = (ijk[a] + s->c.n[a]) % s->c.n[a];
    }
    int n = cell_id(s, ijk);
    if (s->solid[n]) {
        int ip = s->pnb[6 * c + 2 * a + (side > 0)];
        *kind = 2;
        *nbc = -1;
        return s->gh[A][(size_t)ip * s->NV + k];
    }
    *kind = 0;
    *nbc = n;
    return s->f[A][(size_t)n * s->NV + k];
}

/* full van Leer slope of a fluid cell along axis a with ghost substitution */
static double full_slope(const or_state *s, int A, int c, int a, int k)
{
    int kl, kr, nl, nr;
    double fl = nb_value(s, A, c, a, -1, k, &kl, &nl);
    double fr = nb_value(s, A, c, a, +1, k, &kr, &nr);
    double fcv = s->f[A][(size_t)c * s->NV + k];
    return vanleer((fcv - fl) / s->dx[a], (fr - fcv) / s->dx[a]);
}

/* upwind face state on the face of fluid cell c toward side (reconstruction
 * equation of Section 2.2) */
static double face_state(const or_state *s, int A, int c, int a, int side, int k)
{
    double xa = s->xi[3 * k + a];
    double h = s->dx[a];
    if (side * xa > 0.0) return s->f[A][(size_t)c * s->NV + k] + side * full_slope(s, A, c, a, k) * (0.5 * h);
    int kind, n;
    double fv = nb_value(s, A, c, a, side, k, &kind, &n);
    if (kind == 1) return fv; /* outer freestream or wall ghost: zero slope (readings R15, R29) */
    if (kind == 2) {
        int ip = s->pnb[6 * c + 2 * a + (side > 0)];
        return s->fc[A][(size_t)ip * s->NV + k];
    }
    return fv - side * full_slope(s, A, n, a, k) * (0.5 * h);
}

static void update(or_state *s, double dt)
{
    int D = s->D, NV = s->NV;
#pragma omp parallel
    {
        double *g0 = (double *)malloc(sizeof(double) * NV), *g1 = (double *)malloc(sizeof(double) * NV);
#pragma omp for schedule(static)
        for (int c = 0; c < s->Nc; ++c) {
            size_t o = (size_t)c * NV;
            if (s->solid[c]) {
                for (int A = 0; A < s->NA; ++A)
                    for (int k = 0; k < NV; ++k) s->fn[A][o + k] = s->f[A][o + k];
                continue;
            }
            shakhov(s, &s->mom[8 * c], g0, g1);
            double tau = s->tau[c];
            for (int A = 0; A < s->NA; ++A) {
                const double *g = A == 0 ? g0 : g1;
                for (int k = 0; k < NV; ++k) {
                    double div = 0.0;
                    for (int a = 0; a < D; ++a) {
                        double xa = s->xi[3 * k + a];
                        double Fp = xa * face_state(s, A, c, a, +1, k);
                        double Fm = xa * face_state(s, A, c, a, -1, k);
                        div += (Fp - Fm) / s->dx[a];
                    }
                    double fv = s->f[A][o + k];
                    if (s->c.flags & OR_FLAG_IMPLICIT)
                        s->fn[A][o + k] = fv - dt * div; /* transport only (R30) */
                    else
                        s->fn[A][o + k] = fv - dt * div + dt / tau * (g[k] - fv);
                }
            }
        }
        free(g0);
        free(g1);
    }
    for (int A = 0; A < s->NA; ++A) {
        double *t = s->f[A];
        s->f[A] = s->fn[A];
        s->fn[A] = t;
    }
}

/* Semi-implicit collision (reading R30; the paper marches every case with
 * forward Euler).  After the transport step the collision conserves rho, U
 * and T, so the relaxation f = f* + (dt/tau)(g^S - f) is taken at the new
 * time with rho, U, T of the transported state f* and with tau from them.
 * The heat flux of the new state satisfies q = q* + r((1 - Pr) q - q) with
 * r = dt/tau (the Shakhov equilibrium carries (1 - Pr) times the heat flux,
 * Section 2.1), so q = q* / (1 + Pr r), and then f = (f* + r g^S) / (1 + r). */
static void implicit_relax(or_state *s, double dt)
{
    const int NV = s->NV;
#pragma omp parallel
    {
        double *g0 = (double *)malloc(sizeof(double) * NV), *g1 = (double *)malloc(sizeof(double) * NV);
#pragma omp for schedule(static)
        for (int c = 0; c < s->Nc; ++c) {
            if (s->solid[c]) continue;
            const size_t o = (size_t)c * NV;
            double mom[8];
            cell_moments(s, s->f[0] + o, s->NA == 2 ? s->f[1] + o : NULL, mom);
            const double r = dt / relax_time(s, mom[0], mom[4]);
            for (int a = 0; a < 3; ++a) mom[5 + a] /= 1.0 + s->c.Pr * r;
            shakhov(s, mom, g0, g1);
            for (int A = 0; A < s->NA; ++A) {
                const double *g = A == 0 ? g0 : g1;
                for (int k = 0; k < NV; ++k) s->f[A][o + k] = (s->f[A][o + k] + r * g[k]) / (1.0 + r);
            }
        }
        free(g0);
        free(g1);
    }
}

/* advance n forward-Euler steps (Section 4: forward Euler in all cases) */
void or_step(void *h, int n)
{
    or_state *s = (or_state *)h;
    for (int it = 0; it < n; ++it) {
        all_moments(s);
        double dt = time_step(s);
        ib_fill(s);
        if (s->c.outer == OR_WALLS) wall_fill(s);
        if (s->c.outer == OR_SPECULAR) specular_fill(s);
        update(s, dt);
        if (s->c.flags & OR_FLAG_IMPLICIT) implicit_relax(s, dt);
        s->dt = dt;
        s->time += dt;
        s->step++;
    }
}

/* ------------------------------------------------------------------ */
/* outputs                                                             */
/* ------------------------------------------------------------------ */

void or_moments(void *h, double *out)
{
    or_state *s = (or_state *)h;
    all_moments(s);
    memcpy(out, s->mom, sizeof(double) * 8 * s->Nc);
}

void or_tau(void *h, double *out)
{
    or_state *s = (or_state *)h;
    all_moments(s);
    memcpy(out, s->tau, sizeof(double) * s->Nc);
}

double or_next_dt(void *h)
{
    or_state *s = (or_state *)h;
    all_moments(s);
    return time_step(s);
}

void or_clock(void *h, double *out3)
{
    or_state *s = (or_state *)h;
    out3[0] = s->dt;
    out3[1] = s->time;
    out3[2] = (double)s->step;
}

/* body force from the momentum flux through the immersed-boundary faces
 * (reading R16) and drag/lift coefficients; wall records per pair (17
 * doubles): x_w[3], n_w[3], rho_w, p_w, tau_w[3], q_n, C_p, T_s, u_s[3].  With the wall
 * distribution f*_w (at rest) and n into the gas: p_w = sum w (xi.n)^2 f*_w,
 * the shear tau_w = sum w (xi.n) (xi - (xi.n) n) f*_w (the tangential part of
 * the momentum flux through the wall), the normal heat flux q_n = 1/2 sum w
 * (xi.n) (|xi|^2 h + b) (2D reduced; 3D: |xi|^2 f), and the pressure
 * coefficient of Section 4, C_p = 2 (p_w - p_0) / (rho_0 U_0^2) with the
 * freestream p_0 = rho_0 T_0 / 2 = 1/2 and U_0 the freestream speed; T_s and
 * u_s are the temperature and velocity of the gas at the wall point, the
 * moments (Section 2.1 definitions) of f*_w, which Section 4 plots along
 * the body surface */
void or_forces(void *h, double *F3, double *cdcl, double *wall)
{
    or_state *s = (or_state *)h;
    int D = s->D, NV = s->NV;
    ib_fill(s);
    double F[3] = {0, 0, 0};
    for (int ip = 0; ip < s->npairs; ++ip) {
        const or_pair *p = &s->pairs[ip];
        int a = p->axis, side = -p->sign;
        double dS = 1.0;
        for (int b = 0; b < D; ++b)
            if (b != a) dS *= s->dx[b];
        double Fp[3] = {0, 0, 0};
        for (int k = 0; k < NV; ++k) {
            const double *x = &s->xi[3 * k];
            double ff = face_state(s, 0, p->dc, a, side, k);
            double xn = side * x[a];
            for (int b = 0; b < D; ++b) Fp[b] += s->w[k] * x[b] * xn * ff;
        }
        for (int b = 0; b < D; ++b) F[b] += dS * Fp[b];
        if (wall) {
            double pw = 0.0, tau[3] = {0, 0, 0}, qn = 0.0;
            for (int k = 0; k < NV; ++k) {
                const double *x = &s->xi[3 * k];
                double dn = 0.0, x2 = 0.0;
                for (int b = 0; b < D; ++b) {
                    dn += x[b] * p->nw[b];
                    x2 += x[b] * x[b];
                }
                const double fw = s->fw[0][(size_t)ip * NV + k];
                pw += s->w[k] * dn * dn * fw;
                for (int b = 0; b < D; ++b) tau[b] += s->w[k] * dn * (x[b] - dn * p->nw[b]) * fw;
                const double e = x2 * fw + (s->NA == 2 ? s->fw[1][(size_t)ip * NV + k] : 0.0);
                qn += 0.5 * s->w[k] * dn * e;
            }
            double mw[8];
            cell_moments(s, s->fw[0] + (size_t)ip * NV, s->NA == 2 ? s->fw[1] + (size_t)ip * NV : NULL, mw);
            double *wr = &wall[17 * ip];
            for (int b = 0; b < 3; ++b) {
                wr[b] = p->xw[b];
                wr[3 + b] = p->nw[b];
                wr[8 + b] = tau[b];
                wr[14 + b] = mw[1 + b];
            }
            wr[6] = s->rhow[ip];
            wr[7] = pw;
            wr[11] = qn;
            wr[12] = s->Uinf > 0 ? 2.0 * (pw - 0.5) / (s->Uinf * s->Uinf) : NAN;
            wr[13] = mw[4];
        }
    }
    for (int b = 0; b < 3; ++b) F3[b] = F[b];
    double L = 1.0;
    switch (s->c.gkind) {
    case OR_G_CIRCLE:
    case OR_G_ELLIPSE:
        L = 2.0 * s->c.gsize[0];
        break;
    case OR_G_AIRFOIL:
        L = s->c.gsize[0];
        break;
    case OR_G_SPHERE:
        L = M_PI * s->c.gsize[0] * s->c.gsize[0];
        break;
    }
    double qd = 0.5 * 1.0 * s->Uinf * s->Uinf * L;
    cdcl[0] = qd > 0 ? F[0] / qd : NAN;
    cdcl[1] = qd > 0 ? F[1] / qd : NAN;
}

/* ------------------------------------------------------------------ */
/* introspection for tests                                             */
/* ------------------------------------------------------------------ */

void or_info(void *h, int *out)
{
    or_state *s = (or_state *)h;
    int nf = 0;
    for (int c = 0; c < s->Nc; ++c) nf += !s->solid[c];
    out[0] = s->D;
    out[1] = s->Nc;
    out[2] = s->NV;
    out[3] = s->NA;
    out[4] = s->npairs;
    out[5] = nf;
    out[6] = s->nghost;
}

void or_velocity(void *h, double *xi3, double *w)
{
    or_state *s = (or_state *)h;
    memcpy(xi3, s->xi, sizeof(double) * 3 * s->NV);
    memcpy(w, s->w, sizeof(double) * s->NV);
}

void or_freestream(void *h, double *f0, double *f1)
{
    or_state *s = (or_state *)h;
    memcpy(f0, s->fs[0], sizeof(double) * s->NV);
    if (s->NA == 2 && f1) memcpy(f1, s->fs[1], sizeof(double) * s->NV);
}

double or_mu0(void *h) { return ((or_state *)h)->mu0; }

/* threads the OpenMP loops of the oracle use from now on (CPU timing at a
 * given core count) */
void or_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

/* threads the OpenMP loops of the oracle use */
int or_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}

/* integer index sets: cell solid flags; per pair gc, dc, ac, axis, sign, ns,
 * then 26 surface-cell indices (-1 padded); per pair velocity classes */
void or_index_sets(void *h, uint8_t *solid, int32_t *pint, uint8_t *cls)
{
    or_state *s = (or_state *)h;
    memcpy(solid, s->solid, s->Nc);
    for (int ip = 0; ip < s->npairs; ++ip) {
        const or_pair *p = &s->pairs[ip];
        int32_t *o = &pint[32 * ip];
        o[0] = p->gc;
        o[1] = p->dc;
        o[2] = p->ac;
        o[3] = p->axis;
        o[4] = p->sign;
        o[5] = p->ns;
        for (int j = 0; j < 26; ++j) o[6 + j] = j < p->ns ? p->sc[j] : -1;
        if (cls) memcpy(cls + (size_t)ip * s->NV, p->cls, s->NV);
    }
}

/* per pair: xw[3], nw[3], xsp[3]; per pair and node: incident measure */
void or_pair_geometry(void *h, double *g9, double *wg)
{
    or_state *s = (or_state *)h;
    for (int ip = 0; ip < s->npairs; ++ip) {
        const or_pair *p = &s->pairs[ip];
        for (int b = 0; b < 3; ++b) {
            g9[9 * ip + b] = p->xw[b];
            g9[9 * ip + 3 + b] = p->nw[b];
            g9[9 * ip + 6 + b] = p->xsp[b];
        }
        if (wg) memcpy(wg + (size_t)ip * s->NV, p->wg, sizeof(double) * s->NV);
    }
}

/* run the ghost construction on the current state and return its stages,
 * each [NA][npairs*NV]: shifted point, intermediate ghost, incident wall,
 * wall, ghost value, ghost-side face value; plus rho_w per pair */
void or_fill_debug(void *h, double *fsp, double *fgc, double *fiw, double *fw, double *gh, double *fc, double *rhow)
{
    or_state *s = (or_state *)h;
    ib_fill(s);
    size_t np = (size_t)s->npairs * s->NV;
    for (int A = 0; A < s->NA; ++A) {
        memcpy(fsp + A * np, s->fsp[A], np * sizeof(double));
        memcpy(fgc + A * np, s->fgc[A], np * sizeof(double));
        memcpy(fiw + A * np, s->fiw[A], np * sizeof(double));
        memcpy(fw + A * np, s->fw[A], np * sizeof(double));
        memcpy(gh + A * np, s->gh[A], np * sizeof(double));
        memcpy(fc + A * np, s->fc[A], np * sizeof(double));
    }
    memcpy(rhow, s->rhow, sizeof(double) * s->npairs);
}

/* upwind weights of pair ip at node k, [ns] */
int or_weights(void *h, int ip, int k, double *w)
{
    or_state *s = (or_state *)h;
    const or_pair *p = &s->pairs[ip];
    upwind_weights(s, p, &s->xi[3 * k], w);
    return p->ns;
}

/* moments and equilibria of arbitrary single-cell distributions */
void or_cell_moments(void *h, const double *f0, const double *f1, double *out8)
{
    cell_moments((or_state *)h, f0, f1, out8);
}

void or_shakhov(void *h, const double *mom8, double *g0, double *g1) { shakhov((or_state *)h, mom8, g0, g1); }

void or_maxwellian(void *h, double rho, const double *U3, double T, double *g0, double *g1)
{
    maxwellian((or_state *)h, rho, U3, T, g0, g1);
}

/* cut-cell sets and incident measures for an arbitrary unit normal */
void or_cut_sets(void *h, const double *n3, uint8_t *cls, double *wg) { build_cut_sets((or_state *)h, n3, cls, wg); }

/* wall density and wall distribution of a single wall point with normal n
 * for given incident arrays fi0 (h or f), fi1 (b); outputs fw0, fw1 */
double or_wall_distribution(void *h, const double *n3, const double *fi0, const double *fi1, double *fw0,
                            double *fw1)
{
    or_state *s = (or_state *)h;
    int NV = s->NV;
    unsigned char *cls = (unsigned char *)malloc(NV);
    double *wg = (double *)malloc(sizeof(double) * NV);
    build_cut_sets(s, n3, cls, wg);
    double *fi[2] = {(double *)fi0, (double *)fi1};
    double *fs[2] = {(double *)calloc(NV, sizeof(double)), (double *)calloc(NV, sizeof(double))};
    double *fw[2] = {fw0, fw1};
    for (int A = 0; A < s->NA; ++A)
        if (s->c.alpha < 1.0) specular_part(s, n3, fi[A], fs[A]);
    double rw;
    wall_distribution(s, n3, s->c.Uw, cls, wg, fi, fs, 0, &rw, fw);
    free(cls);
    free(wg);
    free(fs[0]);
    free(fs[1]);
    return rw;
}
