// geometry.cpp -- immersed-boundary preprocessing for the HIP library.
//
// Written independently of the CPU oracle.  Only the predicates that decide
// integer index sets are alike by necessity (cell centres lo + (i + 1/2) dx,
// the level-set expressions, velocity nodes about the box centre, dual-cell
// edges, corner dot products and the 1e-12 snap): both sides must take the
// same decisions bit for bit.  Intersect points use closed-form roots,
// cut-cell measures a clamped-linear integral (2D) and Gauss-Legendre
// integration of exact cross-sections (3D).  Compile without FP contraction.
#include "geometry.hpp"

#include "ibdvm.h"

#include <algorithm>
#include <cmath>

namespace ibdvm {

namespace {

struct Shape {
    const Problem &p;
    explicit Shape(const Problem &pp) : p(pp) {}

    void body(const double x[3], double &xp, double &yp) const
    {
        double dx = x[0] - p.gcen[0], dy = x[1] - p.gcen[1];
        double ca = std::cos(p.aoa), sa = std::sin(p.aoa);
        xp = dx * ca - dy * sa;
        yp = dx * sa + dy * ca;
    }

    static double yt(double t, double X)
    {
        return 5.0 * t * (0.2969 * std::sqrt(X) - 0.1260 * X - 0.3516 * X * X + 0.2843 * X * X * X - 0.1036 * X * X * X * X);
    }

    static double dyt(double t, double X)
    {
        X = std::max(X, 1e-12);
        return 5.0 * t * (0.2969 * 0.5 / std::sqrt(X) - 0.1260 - 2.0 * 0.3516 * X + 3.0 * 0.2843 * X * X - 4.0 * 0.1036 * X * X * X);
    }

    // level set, negative inside the body
    double phi(const double x[3]) const
    {
        switch (p.gkind) {
        case 1: {
            double dx = x[0] - p.gcen[0], dy = x[1] - p.gcen[1];
            return dx * dx + dy * dy - p.gsize[0] * p.gsize[0];
        }
        case 4: {
            double dx = x[0] - p.gcen[0], dy = x[1] - p.gcen[1], dz = x[2] - p.gcen[2];
            return dx * dx + dy * dy + dz * dz - p.gsize[0] * p.gsize[0];
        }
        case 2: {
            double xp, yp;
            body(x, xp, yp);
            double u = xp / p.gsize[0], v = yp / p.gsize[1];
            return u * u + v * v - 1.0;
        }
        case 3: {
            double xp, yp;
            body(x, xp, yp);
            double ch = p.gsize[0];
            double X = xp / ch, Y = yp / ch;
            if (X < 0.0) return ch * std::sqrt(X * X + Y * Y);
            if (X > 1.0) return ch * std::sqrt((X - 1.0) * (X - 1.0) + Y * Y);
            return ch * (std::fabs(Y) - yt(p.gsize[1], X));
        }
        default:
            return 1.0;
        }
    }

    void normal(const double x[3], double nrm[3]) const
    {
        double g[3] = {0, 0, 0};
        if (p.gkind == 1 || p.gkind == 4) {
            for (int a = 0; a < p.dim; ++a) g[a] = x[a] - p.gcen[a];
        } else if (p.gkind == 2 || p.gkind == 3) {
            double xp, yp, gx, gy;
            body(x, xp, yp);
            if (p.gkind == 2) {
                gx = xp / (p.gsize[0] * p.gsize[0]);
                gy = yp / (p.gsize[1] * p.gsize[1]);
            } else {
                double ch = p.gsize[0], X = xp / ch, Y = yp / ch;
                if (X <= 0.0) {
                    gx = X;
                    gy = Y;
                } else if (X >= 1.0) {
                    gx = X - 1.0;
                    gy = Y;
                } else {
                    gx = -dyt(p.gsize[1], X);
                    gy = Y >= 0.0 ? 1.0 : -1.0;
                }
            }
            double ca = std::cos(p.aoa), sa = std::sin(p.aoa);
            g[0] = gx * ca + gy * sa;
            g[1] = -gx * sa + gy * ca;
        }
        double m = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        for (int a = 0; a < 3; ++a) nrm[a] = a < p.dim ? g[a] / m : 0.0;
    }

    // wall crossing on the axis segment from the ghost centre xg (inside)
    // toward the donor centre at xg[a] + sign*dx
    double root(const double xg[3], int a, double xd_a) const
    {
        double lo = std::min(xg[a], xd_a), hi = std::max(xg[a], xd_a);
        double t;
        if (p.gkind == 1 || p.gkind == 4) {
            double rest = 0.0;
            for (int b = 0; b < p.dim; ++b)
                if (b != a) rest += (xg[b] - p.gcen[b]) * (xg[b] - p.gcen[b]);
            double s = xd_a > xg[a] ? 1.0 : -1.0;
            t = p.gcen[a] + s * std::sqrt(std::max(0.0, p.gsize[0] * p.gsize[0] - rest));
        } else if (p.gkind == 2) {
            // phi(x0 + tau e_a) = A tau^2 + B tau + C with body-frame rotation
            double ca = std::cos(p.aoa), sa = std::sin(p.aoa);
            double d0x = (a == 0 ? 0.0 : xg[0]) - p.gcen[0], d0y = (a == 1 ? 0.0 : xg[1]) - p.gcen[1];
            double ex = a == 0 ? 1.0 : 0.0, ey = a == 1 ? 1.0 : 0.0;
            double px0 = d0x * ca - d0y * sa, py0 = d0x * sa + d0y * ca;
            double pxe = ex * ca - ey * sa, pye = ex * sa + ey * ca;
            double ia = 1.0 / (p.gsize[0] * p.gsize[0]), ib = 1.0 / (p.gsize[1] * p.gsize[1]);
            double A = pxe * pxe * ia + pye * pye * ib;
            double B = 2.0 * (px0 * pxe * ia + py0 * pye * ib);
            double C = px0 * px0 * ia + py0 * py0 * ib - 1.0;
            double disc = std::sqrt(std::max(0.0, B * B - 4.0 * A * C));
            double q = -0.5 * (B + (B >= 0 ? disc : -disc));
            double r1 = q / A, r2 = (q != 0.0) ? C / q : r1;
            // the crossing inside the segment (closest to its midpoint)
            double mid = 0.5 * (lo + hi);
            t = std::fabs(r1 - mid) < std::fabs(r2 - mid) ? r1 : r2;
        } else {
            // airfoil: sign-change search by interval halving
            double x[3] = {xg[0], xg[1], xg[2]};
            double in = xg[a], out = xd_a;
            for (int it = 0; it < 200; ++it) {
                double m = in + 0.5 * (out - in);
                if (m == in || m == out) break;
                x[a] = m;
                if (phi(x) < 0.0)
                    in = m;
                else
                    out = m;
            }
            t = out;
        }
        return std::min(hi, std::max(lo, t));
    }
};

// exact integral of clamp(a0 + a1 x, 0, L) over [x0, x1]: the integrand is
// piecewise linear with breaks where it reaches 0 or L
double clamped_linear_integral(double a0, double a1, double L, double x0, double x1)
{
    double br[4] = {x0, x1, x0, x0};
    int m = 2;
    if (a1 != 0.0) {
        double z0 = -a0 / a1, zL = (L - a0) / a1;
        if (z0 > x0 && z0 < x1) br[m++] = z0;
        if (zL > x0 && zL < x1) br[m++] = zL;
    }
    std::sort(br, br + m);
    auto g = [&](double x) { return std::min(L, std::max(0.0, a0 + a1 * x)); };
    double s = 0.0;
    for (int i = 0; i + 1 < m; ++i)
        if (br[i + 1] > br[i]) s += 0.5 * (br[i + 1] - br[i]) * (g(br[i]) + g(br[i + 1]));
    return s;
}

// area of {v in [x0,x1]x[y0,y1] : na*vx + nb*vy <= c}, integrating along the
// axis whose normal component is smaller in magnitude
double area2(double x0, double x1, double y0, double y1, double na, double nb, double c)
{
    if (std::fabs(na) > std::fabs(nb)) return area2(y0, y1, x0, x1, nb, na, c);
    double L = y1 - y0;
    if (nb == 0.0) return c >= 0.0 ? (x1 - x0) * L : 0.0;
    // nb > 0: vy <= (c - na vx)/nb ; nb < 0: vy >= (c - na vx)/nb
    if (nb > 0.0) return clamped_linear_integral(c / nb - y0, -na / nb, L, x0, x1);
    return clamped_linear_integral(y1 - c / nb, na / nb, L, x0, x1);
}

}  // namespace

double incident_measure(int dim, const double e0[3], const double e1[3], const double n[3])
{
    if (dim == 2) return area2(e0[0], e1[0], e0[1], e1[1], n[0], n[1], 0.0);
    // integrate the exact cross-section area along the axis q with the
    // smallest normal component; the area is quadratic between the values of
    // v_q where the cutting line passes a corner, 3-point Gauss-Legendre is
    // exact there
    int q = 0;
    for (int a = 1; a < 3; ++a)
        if (std::fabs(n[a]) < std::fabs(n[q])) q = a;
    int a = (q + 1) % 3, b = (q + 2) % 3;
    auto A = [&](double vq) { return area2(e0[a], e1[a], e0[b], e1[b], n[a], n[b], -n[q] * vq); };
    if (n[q] == 0.0) return A(0.0) * (e1[q] - e0[q]);
    std::vector<double> br = {e0[q], e1[q]};
    for (int ca = 0; ca < 2; ++ca)
        for (int cb = 0; cb < 2; ++cb) {
            double va = ca ? e1[a] : e0[a], vb = cb ? e1[b] : e0[b];
            double z = -(n[a] * va + n[b] * vb) / n[q];
            if (z > e0[q] && z < e1[q]) br.push_back(z);
        }
    std::sort(br.begin(), br.end());
    const double gx = std::sqrt(3.0 / 5.0);
    double V = 0.0;
    for (size_t i = 0; i + 1 < br.size(); ++i) {
        double h = 0.5 * (br[i + 1] - br[i]), m = 0.5 * (br[i + 1] + br[i]);
        if (h <= 0.0) continue;
        V += h * (5.0 / 9.0 * A(m - gx * h) + 8.0 / 9.0 * A(m) + 5.0 / 9.0 * A(m + gx * h));
    }
    return V;
}

int build_geometry(const Problem &p, Geometry &g, std::string &err)
{
    const int D = p.dim;
    g.D = D;
    g.Nc = 1;
    g.NV = 1;
    for (int a = 0; a < D; ++a) {
        g.Nc *= p.n[a];
        g.NV *= p.vn[a];
        g.dx[a] = (p.hi[a] - p.lo[a]) / (double)p.n[a];
    }
    // velocity nodes about the box centre (exactly antisymmetric for a
    // symmetric box) with midpoint or trapezoid weights and dual cells
    // x +- h/2 clipped to the box; or the stretched grid: the image under
    // x(u) = V sinh(beta u)/sinh(beta) of the midpoint grid of u in [-1, 1]
    // and of its cells, u = m/N with an integer m so that nodes and cell
    // faces are exactly antisymmetric
    for (int a = 0; a < D; ++a) {
        int N = p.vn[a];
        g.xa[a].resize(N);
        g.wa[a].resize(N);
        g.ea0[a].resize(N);
        g.ea1[a].resize(N);
        if (p.rule == 3) {
            // refined grid: density 1 + A sum_c exp(-((x - c)/w)^2) over the
            // centres 0 and c_a; its cumulative from -V in closed form (erf)
            // is inverted by bisection at u = m/N; an axis with the one
            // centre at 0 has an even density, and its negative half is the
            // mirror of the positive one
            const double V = p.vhi[a], A = p.vref_amp, w = p.vref_width;
            const double cen[2] = {0.0, p.vref_centre[a]};
            const int nc = p.vref_centre[a] != 0.0 ? 2 : 1;
            auto cum = [&](double x) {
                double s = x + V;
                for (int i = 0; i < nc; ++i)
                    s += A * w * 0.5 * std::sqrt(M_PI) * (std::erf((x - cen[i]) / w) - std::erf((-V - cen[i]) / w));
                return s;
            };
            const double total = cum(V);
            auto inv = [&](int k) {  // the point where the normalised cumulative reaches k/N
                if (k <= -N) return -V;
                if (k >= N) return V;
                const double t = 0.5 * ((double)k / (double)N + 1.0) * total;
                double lo = -V, hi = V;
                for (int it = 0; it < 200; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (mid == lo || mid == hi) break;
                    if (cum(mid) < t)
                        lo = mid;
                    else
                        hi = mid;
                }
                return 0.5 * (lo + hi);
            };
            auto map = [&](int k) { return nc == 1 && k == 0 ? 0.0 : (nc == 1 && k < 0 ? -inv(-k) : inv(k)); };
            g.dxi[a] = 0.0;
            for (int i = 0; i < N; ++i) {
                g.xa[a][i] = map(2 * i + 1 - N);
                g.ea0[a][i] = map(2 * i - N);
                g.ea1[a][i] = map(2 * i + 2 - N);
                if (p.vweights) {
                    // the map's derivative total / (2 rho(x)) times the u-cell width 2/N
                    double rho = 1.0;
                    for (int c = 0; c < nc; ++c) {
                        const double z = (g.xa[a][i] - cen[c]) / w;
                        rho += A * std::exp(-z * z);
                    }
                    g.wa[a][i] = total / ((double)N * rho);
                } else {
                    g.wa[a][i] = g.ea1[a][i] - g.ea0[a][i];
                }
            }
            continue;
        }
        if (p.rule == 2) {
            const double V = p.vhi[a], beta = p.vstretch;
            auto map = [&](int m) { return V * std::sinh(beta * ((double)m / (double)N)) / std::sinh(beta); };
            g.dxi[a] = 0.0;
            for (int i = 0; i < N; ++i) {
                g.xa[a][i] = map(2 * i + 1 - N);
                g.ea0[a][i] = map(2 * i - N);
                g.ea1[a][i] = map(2 * i + 2 - N);
                // Jacobian weights: V beta cosh(beta u) / sinh(beta) times 2/N
                g.wa[a][i] = p.vweights ? V * beta * std::cosh(beta * ((double)(2 * i + 1 - N) / (double)N)) /
                                              std::sinh(beta) * (2.0 / (double)N)
                                        : g.ea1[a][i] - g.ea0[a][i];
            }
            continue;
        }
        bool trap = p.rule == 1;
        double h = trap ? (p.vhi[a] - p.vlo[a]) / (double)(N - 1) : (p.vhi[a] - p.vlo[a]) / (double)N;
        double c = 0.5 * (p.vlo[a] + p.vhi[a]);
        g.dxi[a] = h;
        for (int i = 0; i < N; ++i) {
            g.xa[a][i] = c + ((double)i - 0.5 * (double)(N - 1)) * h;
            g.wa[a][i] = (trap && (i == 0 || i == N - 1)) ? 0.5 * h : h;
            g.ea0[a][i] = std::max(p.vlo[a], g.xa[a][i] - 0.5 * h);
            g.ea1[a][i] = std::min(p.vhi[a], g.xa[a][i] + 0.5 * h);
        }
    }
    g.xi.assign((size_t)3 * g.NV, 0.0);
    g.w.assign(g.NV, 1.0);
    for (int k = 0; k < g.NV; ++k) {
        int r = k;
        for (int a = 0; a < D; ++a) {
            int i = r % p.vn[a];
            r /= p.vn[a];
            g.xi[3 * k + a] = g.xa[a][i];
            g.w[k] *= g.wa[a][i];
        }
    }

    Shape shape(p);
    auto centre = [&](int a, int i) { return p.lo[a] + ((double)i + 0.5) * g.dx[a]; };
    int stride[3] = {1, p.n[0], p.n[0] * p.n[1]};
    auto decompose = [&](int c, int ijk[3]) {
        ijk[0] = c % p.n[0];
        ijk[1] = (c / p.n[0]) % p.n[1];
        ijk[2] = D == 3 ? c / (p.n[0] * p.n[1]) : 0;
    };

    // classification: solid iff the level set is negative at the centre
    g.cflag.assign(g.Nc, 0);
    for (int c = 0; c < g.Nc; ++c) {
        int ijk[3];
        decompose(c, ijk);
        double x[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) x[a] = centre(a, ijk[a]);
        if (p.gkind != 0 && shape.phi(x) < 0.0) {
            g.cflag[c] = CF_SOLID;
            for (int a = 0; a < D; ++a)
                if (ijk[a] < 3 || ijk[a] > p.n[a] - 4) {
                    err = "body closer than 3 cells to the outer boundary";
                    return 2;
                }
        }
    }
    auto solid = [&](int c) { return (g.cflag[c] & CF_SOLID) != 0; };
    g.nfluid = 0;
    for (int c = 0; c < g.Nc; ++c) g.nfluid += !solid(c);

    // cells whose axis stencil (+-1, +-2) leaves the plain interior
    for (int c = 0; c < g.Nc; ++c) {
        if (solid(c)) continue;
        int ijk[3];
        decompose(c, ijk);
        bool near = false;
        for (int a = 0; a < D && !near; ++a)
            for (int o = -2; o <= 2 && !near; ++o) {
                if (o == 0) continue;
                int i = ijk[a] + o;
                if (i < 0 || i >= p.n[a]) {
                    near = true;
                    break;
                }
                if (solid(c + o * stride[a])) near = true;
            }
        if (near) g.cflag[c] |= CF_NEAR;
        for (int a = 0; a < D; ++a)
            for (int s = 0; s < 2; ++s) {
                int i = ijk[a] + (s ? 1 : -1);
                if (i >= 0 && i < p.n[a] && solid(c + (s ? 1 : -1) * stride[a])) g.cflag[c] |= (uint8_t)(CF_XM << (2 * a + s));
            }
    }

    // ghost-donor pairs in ghost order, then axis, then side
    g.pnb.assign((size_t)6 * g.Nc, -1);
    g.pairs.clear();
    g.nghost = 0;
    for (int c = 0; c < g.Nc; ++c) {
        if (!solid(c)) continue;
        int ijk[3];
        decompose(c, ijk);
        bool ghost = false;
        for (int a = 0; a < D; ++a)
            for (int sg = -1; sg <= 1; sg += 2) {
                int d = c + sg * stride[a];
                if (solid(d)) continue;
                ghost = true;
                PairGeom pr{};
                pr.gc = c;
                pr.dc = d;
                pr.axis = a;
                pr.sign = sg;
                double xg[3] = {0, 0, 0};
                for (int b = 0; b < D; ++b) xg[b] = centre(b, ijk[b]);
                double xd_a = centre(a, ijk[a] + sg);
                for (int b = 0; b < 3; ++b) pr.xw[b] = xg[b];
                pr.xw[a] = shape.root(xg, a, xd_a);
                shape.normal(pr.xw, pr.nw);
                for (int b = 0; b < 3; ++b) pr.xsp[b] = pr.xw[b];
                pr.xsp[a] = pr.xw[a] + 0.5 * (xd_a - xg[a]);
                int ai = ijk[a] + 2 * sg;
                // auxiliary cell next to the donor (none with the no-donor-slope ablation)
                const bool no_aux = (p.flags & IBDVM_FLAG_NO_AUX_SLOPE) != 0;
                pr.ac = (ai >= 0 && ai < p.n[a] && !solid(c + 2 * sg * stride[a]) && !no_aux) ? c + 2 * sg * stride[a]
                                                                                              : -1;
                // wall velocity at the intersect point: translation plus rotation about the centre
                {
                    double r[3] = {0, 0, 0};
                    for (int b = 0; b < D; ++b) r[b] = pr.xw[b] - p.gcen[b];
                    const double *O = p.Ow;
                    const double rot[3] = {O[1] * r[2] - O[2] * r[1], O[2] * r[0] - O[0] * r[2], O[0] * r[1] - O[1] * r[0]};
                    for (int b = 0; b < 3; ++b) pr.uw[b] = b < D ? p.Uw[b] + rot[b] : 0.0;
                }
                // surface cells: fluid members of the Moore neighbourhood
                pr.ns = 0;
                int zr = D == 3 ? 1 : 0;
                for (int dz = -zr; dz <= zr; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dxo = -1; dxo <= 1; ++dxo) {
                            if (!dxo && !dy && !dz) continue;
                            int off[3] = {dxo, dy, dz};
                            int m[3];
                            bool inside = true;
                            for (int b = 0; b < 3; ++b) {
                                m[b] = ijk[b] + off[b];
                                if (b < D && (m[b] < 0 || m[b] >= p.n[b])) inside = false;
                            }
                            if (!inside) continue;
                            int mc = m[0] + p.n[0] * (m[1] + p.n[1] * (D == 3 ? m[2] : 0));
                            if (solid(mc)) continue;
                            int j = pr.ns++;
                            pr.sc[j] = mc;
                            double len = 0.0;
                            for (int b = 0; b < 3; ++b) {
                                pr.r[j][b] = b < D ? centre(b, m[b]) - xg[b] : 0.0;
                                len += pr.r[j][b] * pr.r[j][b];
                            }
                            len = std::sqrt(len);
                            for (int b = 0; b < 3; ++b) pr.rh[j][b] = pr.r[j][b] / len;
                            for (int b = 0; b < 3; ++b)
                                for (int s2 = 0; s2 < 2; ++s2) {
                                    pr.snb[j][b][s2] = -1;
                                    if (b >= D) continue;
                                    int i2 = m[b] + (s2 ? 1 : -1);
                                    if (i2 < 0 || i2 >= p.n[b]) continue;
                                    int nc = mc + (s2 ? 1 : -1) * stride[b];
                                    if (!solid(nc)) pr.snb[j][b][s2] = nc;
                                }
                        }
                g.pnb[(size_t)6 * d + 2 * a + (sg < 0 ? 1 : 0)] = (int)g.pairs.size();
                g.pairs.push_back(pr);
            }
        g.nghost += ghost;
    }

    // velocity-space cut cells per pair (plane xi.n_w = 0)
    const size_t np = g.pairs.size();
    g.cls.assign(np * g.NV, 0);
    g.wg.assign(np * g.NV, 0.0);
    for (size_t ip = 0; ip < np; ++ip) {
        const double *n = g.pairs[ip].nw;
        for (int k = 0; k < g.NV; ++k) {
            int id[3] = {0, 0, 0};
            int r = k;
            for (int a = 0; a < D; ++a) {
                id[a] = r % p.vn[a];
                r /= p.vn[a];
            }
            double e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
            for (int a = 0; a < D; ++a) {
                e0[a] = g.ea0[a][id[a]];
                e1[a] = g.ea1[a][id[a]];
            }
            double dmin = INFINITY, dmax = -INFINITY, vmax = 0.0;
            for (int corner = 0; corner < (1 << D); ++corner) {
                double dd = 0.0, rr = 0.0;
                for (int a = 0; a < D; ++a) {
                    double v = (corner >> a & 1) ? e1[a] : e0[a];
                    dd += v * n[a];
                    rr += v * v;
                }
                dmin = std::min(dmin, dd);
                dmax = std::max(dmax, dd);
                vmax = std::max(vmax, std::sqrt(rr));
            }
            double eps = 1e-12 * vmax, dn = 0.0;
            for (int a = 0; a < D; ++a) dn += g.xi[3 * k + a] * n[a];
            bool cut = dmin < -eps && dmax > eps && !(p.flags & 1u);
            size_t o = ip * g.NV + k;
            if (!cut) {
                g.cls[o] = dn <= 0.0 ? VC_GAS : VC_SOLID;
                g.wg[o] = dn <= 0.0 ? g.w[k] : 0.0;
            } else {
                g.cls[o] = dn <= 0.0 ? VC_CUT_G : VC_CUT_S;
                g.wg[o] = incident_measure(D, e0, e1, n);
                if (p.vweights) {
                    // the incident fraction of the dual cell, of the node's weight
                    double vol = 1.0;
                    for (int a = 0; a < D; ++a) vol *= e1[a] - e0[a];
                    g.wg[o] = g.wg[o] / vol * g.w[k];
                }
            }
        }
    }
    return 0;
}

}  // namespace ibdvm
