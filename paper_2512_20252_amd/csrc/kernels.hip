// kernels.hip -- gfx950 kernels of the immersed-boundary Shakhov-DVM step
// (arXiv 2512.20252).  The velocity node index is innermost in memory, so a
// wavefront's 64 lanes read and write contiguous 512-byte (FP64) or 256-byte
// (FP32) runs of one cell's distribution.
//
//   k_update2d  Section 2.2 upwind MUSCL fluxes with the van Leer limiter,
//   k_update3d  Shakhov relaxation (Sections 2.1, 4), forward Euler; each
//               workgroup marches a tile of grid columns along y (2D) or z
//               (3D) and emits partial moments of the new state per (cell,
//               velocity chunk).
//   k_fill_*    Section 3.2.1 ghost construction with the upwind weights of
//               3.2.2 and the cut-cell wall density/distribution of 3.2.3,
//               over (ghost-donor pair, node chunk) workgroups in three
//               phases; the first launch also finishes the per-cell moments
//               and tau_min in its other workgroups.
//   k_force     momentum flux through the immersed-boundary faces.
//
// Moments of the new state are accumulated about the old bulk velocity U^n
// (peculiar velocity c = xi - U^n, already formed for the equilibrium), so
// the heat flux of the new state follows from shifted raw moments without a
// second pass over the distribution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "device.hpp"
#include "launch.hpp"

namespace ibdvm {

namespace {

constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// van Leer limiter in difference form: (sign s1 + sign s2)|s1||s2|/(|s1|+|s2|)
template <typename T>
__device__ __forceinline__ T vanleer(T s1, T s2)
{
    if ((s1 > T(0) && s2 > T(0)) || (s1 < T(0) && s2 < T(0))) return T(2) * s1 * (s2 / (s1 + s2));
    return T(0);
}

// 2D FP32 storage holds f minus a reference d.fr: by default the
// freestream Maxwellian, so that its rounding is relative to the deviation
// from the freestream (the rounding of a steady state acts like a constant
// source, and the deviation is small over most of the domain), or zero
// (f itself) for flows with near-vacuum regions, where f is far below the
// freestream value and the offset would cancel its digits.  FP64 storage
// and the 3D FP32 form hold f (there the two extra live values per node
// cost the 4 x 4-tile update a fifth of its speed in register spills).
// fref is the offset of a stored value of node k of array A.
template <typename T, typename DR>
__device__ __forceinline__ double fref(const DR &d, int A, int k)
{
    if constexpr (sizeof(T) == 4)
        return d.D == 2 ? d.fr[A][k] : 0.0;
    else
        return 0.0;
}

enum { NB_FLUID = 0, NB_BC = 1, NB_IB = 2 };

// Value seen from fluid cell c (grid coordinates ijk) at c + side e_a:
// fluid value, outer freestream ghost, or the ghost value of the pair whose
// donor is c.  nc returns the fluid neighbour, pr the pair.
template <typename T>
__device__ __forceinline__ T neighbour(const Dev &d, const T *f, int A, int k, int c, const int ijk[3], int a, int side,
                                       int &kind, int &nc, int &pr)
{
    int i = ijk[a] + side;
    if (i < 0 || i >= d.n[a]) {
        if (d.outer != 1) {
            kind = NB_BC;
            nc = -1;
            pr = -1;
            return (T)(d.fs[A][k] - fref<T>(d, A, k));
        }
        i = (i + d.n[a]) % d.n[a];
    }
    int n = c + (i - ijk[a]) * d.stride[a];
    if (d.cflag[n] & 1) {
        kind = NB_IB;
        nc = -1;
        pr = d.pnb[6 * c + 2 * a + (side > 0 ? 1 : 0)];
        return (T)(d.ghost[A][(size_t)pr * d.NV + k] - fref<T>(d, A, k));
    }
    kind = NB_FLUID;
    nc = n;
    pr = -1;
    return f[(size_t)n * d.NV + k];
}

// the cell parameters of one fluid cell from its moments; returns tau.
// With the semi-implicit collision the update record's relaxation rate is 0:
// the update then transports only, and the moment finish relaxes.
template <typename DR>
__device__ double write_cell(const DR &d, int c, double rho, const double U[3], double T, const double q[3], int D)
{
    double tau = d.mu0 * pow(T, d.omega) / (0.5 * rho * T);
    const double rate = (d.flags & kFlagImplicit) ? 0.0 : 1.0 / tau;
    double *cp = d.cellp + (size_t)c * kCellWords;
    double A = (D == 2) ? rho / (kPi * T) : rho * pow(kPi * T, -1.5);
    double coef = d.shk / (rho * T * T);
    for (int a = 0; a < 3; ++a) {
        cp[CW_U + a] = U[a];
        cp[CW_S + a] = coef * q[a];
        cp[CW_Q + a] = q[a];
    }
    cp[CW_A] = A;
    cp[CW_INVT] = 1.0 / T;
    cp[CW_TH] = 0.5 * T;
    cp[CW_INVTAU] = 1.0 / tau;
    cp[CW_RHO] = rho;
    cp[CW_T] = T;
    cp[CW_TAU] = tau;
    if (D == 2) {
        double *k2 = d.cellq + (size_t)c * kQWords;
        k2[0] = U[0];
        k2[1] = U[1];
        k2[2] = A;
        k2[3] = 1.0 / T;
        k2[4] = coef * q[0];
        k2[5] = coef * q[1];
        k2[6] = 0.5 * T;
        k2[7] = rate;
    } else {
        // 3D update record: U[3], A, 1/T, s[3], 1/tau (word 9: flag word of the cell above)
        double *k3 = d.cellq + (size_t)c * kQWords;
        k3[0] = U[0];
        k3[1] = U[1];
        k3[2] = U[2];
        k3[3] = A;
        k3[4] = 1.0 / T;
        k3[5] = coef * q[0];
        k3[6] = coef * q[1];
        k3[7] = coef * q[2];
        k3[8] = rate;
    }
    bool bad = !(rho > 0.0) || !(T > 0.0) || !isfinite(rho) || !isfinite(T) || !isfinite(tau);
    if (bad) atomicOr(&d.ctrl->health, 1u);
    return bad ? INFINITY : tau;
}

template <typename DR>
__device__ __forceinline__ void tau_min_commit(const DR &d, int slot, double tau)
{
    // the semi-implicit collision takes no relaxation-time bound on dt: the
    // slot keeps +inf (uniform over the workgroup)
    if (d.flags & kFlagImplicit) return;
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) tau = fmin(tau, __shfl_xor(tau, m, 64));
    if (lane == 0) red[wv] = tau;
    __syncthreads();
    if (threadIdx.x == 0) {
        // positive doubles order as their bit patterns; most workgroups see a
        // smaller minimum already and skip the atomic on the shared word
        const double t = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
        const unsigned long long tb = (unsigned long long)__double_as_longlong(t);
        unsigned long long *w = &d.ctrl->tau_bits[slot];
        if (t < INFINITY && tb < __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(w, tb);
    }
}

// deterministic sum over the 256 threads of a workgroup
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[4];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

// multilinear interpolation on the velocity nodes, zero outside the node hull
template <typename DR>
__device__ double vel_interp(const DR &d, const double *g, const double v[3], int D)
{
    int i0[3] = {0, 0, 0};
    double t[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
        const double *x = d.xa + a * kMaxVn;
        int N = d.vn[a];
        if (v[a] < x[0] || v[a] > x[N - 1]) return 0.0;
        // interval [x_i, x_i+1] holding v: i = the number of interior nodes
        // x_1 .. x_N-2 below v (binary search; the nodes need not be uniform)
        int lo = 1, hi = N - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (x[mid] < v[a])
                lo = mid + 1;
            else
                hi = mid;
        }
        const int i = lo - 1;
        i0[a] = i;
        t[a] = (v[a] - x[i]) / (x[i + 1] - x[i]);
    }
    double acc = 0.0;
    for (int corner = 0; corner < (1 << D); ++corner) {
        double wgt = 1.0;
        int k = 0, mul = 1;
        for (int a = 0; a < D; ++a) {
            int up = corner >> a & 1;
            wgt *= up ? t[a] : 1.0 - t[a];
            k += (i0[a] + up) * mul;
            mul *= d.vn[a];
        }
        acc += wgt * g[k];
    }
    return acc;
}

// ---------------------------------------------------------------- ghost fill
//
// The fill of one ghost-donor pair runs over (pair, chunk of kFillChunk
// nodes) workgroups in three phases, one launch each: (1) the shifted-point
// and incident distributions and the partial incident flux of the wall
// density balance; (2) with alpha < 1 only, the partial flux of the specular
// part, which interpolates the incident distribution of the whole pair;
// (3) the wall density from all partials, the wall distribution, the ghost
// value and the ghost-side face value.

template <typename DR>
__device__ __forceinline__ int fill_chunks(const DR &d) { return (d.NV + kFillChunk - 1) / kFillChunk; }

// reflected node velocity xi - 2 (xi . n) n and the normal component xi . n
template <int D, typename DR>
__device__ __forceinline__ double reflect(const DR &d, int k, const double nw[3], double v[3])
{
    double dn = 0.0;
    for (int b = 0; b < D; ++b) dn += d.xi[b][k] * nw[b];
    for (int b = 0; b < 3; ++b) v[b] = b < D ? d.xi[b][k] - 2.0 * dn * nw[b] : 0.0;
    return dn;
}

template <int D, typename T, typename DR>
__device__ void fill_incident(const DR &d, int cur, int p, int chunk)
{
    const DPair &P = d.pairs[p];
    const int dc = P.dc, ac = P.ac, ns = P.ns;
    const double ygc = P.ygc, ydc = P.ydc, yac = P.yac, yw = P.yw, ysp = P.ysp;
    const size_t po = (size_t)p * d.NV;
    const int NV = d.NV, k = chunk * kFillChunk + threadIdx.x;
    const bool uniform = (d.flags & 2u) != 0;  // NO_UPWIND ablation
    const bool naive = (d.flags & kFlagNaive) != 0;
    double num = 0.0;
    if (k < NV) {
        double xk[3] = {0, 0, 0}, x2 = 0.0;
        for (int b = 0; b < D; ++b) {
            xk[b] = d.xi[b][k];
            x2 += xk[b] * xk[b];
        }
        // upwind weights of the surface cells: w_j proportional to max(0, -xi . r_j)^2
        const double thr = 1e-12 * sqrt(x2);
        auto upw = [&](int j) {
            double dd = 0.0;
            for (int b = 0; b < D; ++b) dd += xk[b] * P.rh[j][b];
            if (fabs(dd) <= thr) dd = 0.0;
            const double m = dd < 0.0 ? -dd : 0.0;
            return m * m;
        };
        double sum = 0.0;
        for (int j = 0; j < ns; ++j) sum += upw(j);
        for (int A = 0; A < d.NA; ++A) {
            const T *f = (const T *)d.f[cur][A];
            const double rf = fref<T>(d, A, k);
            // 1. shifted point from the donor and the auxiliary-cell slope
            const double fdc = (double)f[(size_t)dc * NV + k] + rf;
            const double sdc = ac >= 0 ? ((double)f[(size_t)ac * NV + k] + rf - fdc) / (yac - ydc) : 0.0;
            const double fspv = fdc + sdc * (ysp - ydc);
            // 2. upwind-weighted interpolation from the surface cells (the
            // naive ablation of Section 3.3.3: linear extrapolation of donor
            // and auxiliary cell along the axis instead)
            double fgc = naive ? fdc + sdc * (ygc - ydc) : 0.0;
            for (int j = 0; j < ns && !naive; ++j) {
                const double wj = (uniform || sum == 0.0) ? 1.0 / ns : upw(j) / sum;
                const int sj = P.sc[j];
                const double fj = (double)f[(size_t)sj * NV + k] + rf;
                double sr = 0.0;
                for (int b = 0; b < D; ++b) {
                    const int L = P.snb[j][b][0], R = P.snb[j][b][1];
                    double sg = 0.0;
                    if (L >= 0 && R >= 0)
                        sg = vanleer(fj - ((double)f[(size_t)L * NV + k] + rf), ((double)f[(size_t)R * NV + k] + rf) - fj) *
                             d.inv_dx[b];
                    else if (R >= 0)
                        sg = (((double)f[(size_t)R * NV + k] + rf) - fj) * d.inv_dx[b];
                    else if (L >= 0)
                        sg = (fj - ((double)f[(size_t)L * NV + k] + rf)) * d.inv_dx[b];
                    sr += sg * P.r[j][b];
                }
                fgc += wj * (fj - sr);
            }
            // 3. incident distribution at the intersect point
            double fiw = fspv + (fgc - fspv) / (ygc - ysp) * (yw - ysp);
            if (fiw < 0.0) fiw = 0.0;  // R28: distributions are non-negative
            d.fiw[A][po + k] = fiw;
            d.fsp[A][po + k] = fspv;
            if (A == 0) {
                double dn = 0.0;
                for (int b = 0; b < D; ++b) dn += xk[b] * P.nw[b];
                const int cl = d.cls[po + k];
                const double wt = cl == 0 ? d.w[k] : (cl >= 2 ? d.wg[po + k] : 0.0);
                num = wt * dn * fiw;
            }
        }
    }
    num = block_sum(num);
    if (threadIdx.x == 0) d.fillpart[((size_t)p * fill_chunks(d) + chunk) * 2] = num;
}

template <int D, typename DR>
__device__ void fill_specular(const DR &d, int p, int chunk)
{
    const DPair &P = d.pairs[p];
    const size_t po = (size_t)p * d.NV;
    const int k = chunk * kFillChunk + threadIdx.x;
    double num = 0.0;
    if (k < d.NV) {
        const int cl = d.cls[po + k];
        if (cl != 0) {
            double v[3];
            const double dn = reflect<D>(d, k, P.nw, v);
            const double fsv = vel_interp(d, d.fiw[0] + po, v, D);
            const double ws = cl == 1 ? d.w[k] : d.w[k] - d.wg[po + k];
            num = (1.0 - d.alpha) * ws * dn * fsv;
        }
    }
    num = block_sum(num);
    if (threadIdx.x == 0) d.fillpart[((size_t)p * fill_chunks(d) + chunk) * 2 + 1] = num;
}

template <int D, typename DR>
__device__ void fill_ghost(const DR &d, int p, int chunk)
{
    const DPair &P = d.pairs[p];
    const double ygc = P.ygc, yw = P.yw, ysp = P.ysp, yface = P.yface;
    const size_t po = (size_t)p * d.NV;
    const int nfc = fill_chunks(d), k = chunk * kFillChunk + threadIdx.x;
    const double al = d.alpha;
    // wall density: zero net mass flux through the wall (the same sum in every workgroup)
    double num = 0.0;
    for (int c = 0; c < nfc; ++c) num += d.fillpart[((size_t)p * nfc + c) * 2];
    if (al < 1.0)
        for (int c = 0; c < nfc; ++c) num += d.fillpart[((size_t)p * nfc + c) * 2 + 1];
    const double rw = al > 0.0 ? -num / (al * P.den) : 0.0;
    if (chunk == 0 && threadIdx.x == 0) d.rhow[p] = rw;
    if (k >= d.NV) return;
    const int cl = d.cls[po + k];
    double v[3] = {0, 0, 0};
    if (al < 1.0 && cl != 0) reflect<D>(d, k, P.nw, v);
    for (int A = 0; A < d.NA; ++A) {
        const double fi = d.fiw[A][po + k];
        const double fsv = (al < 1.0 && cl != 0) ? vel_interp(d, d.fiw[A] + po, v, D) : 0.0;
        const double Hw = (d.hwp ? d.hwp[po + k] : d.hw[k]) * (A == 1 ? 0.5 * d.Tw : 1.0);
        const double fr = al * rw * Hw + (1.0 - al) * fsv;
        const double fw = cl == 0 ? fi : (cl == 1 ? fr : (d.wg[po + k] * fi + (d.w[k] - d.wg[po + k]) * fr) / d.w[k]);
        const double fspv = d.fsp[A][po + k];
        const double sig = (fw - fspv) / (yw - ysp);
        const double gv = fspv + sig * (ygc - ysp);
        // R28: ghost and face values stay non-negative; with the face limit
        // the face value goes no further than the wall value when the face
        // lies beyond the wall
        double t = (yface - ysp) / (yw - ysp);
        if ((d.flags & kFlagFaceLimit) && t > 1.0) t = 1.0;
        const double fv = fspv + (fw - fspv) * t;
        d.ghost[A][po + k] = gv < 0.0 ? 0.0 : gv;
        d.face[A][po + k] = fv < 0.0 ? 0.0 : fv;
        d.fwall[A][po + k] = fw;
    }
}

// ---------------------------------------------------------------- moments
// rho, U, T, q of a cell from its moment sums about Uref: S = m0, m1[D],
// m2, m3[D], M (upper triangle), with m2 and m3 over c^2 h + b in 2D (the
// record the update writes per node chunk)
template <int D>
__device__ __forceinline__ void moments_from_sums(const double *S, const double Uref[3], double &rho, double U[3],
                                                  double &T, double q[3])
{
    double m1[3] = {0, 0, 0}, m3[3] = {0, 0, 0}, M[3][3] = {};
    const double m0 = S[0];
    for (int a = 0; a < D; ++a) {
        m1[a] = S[1 + a];
        m3[a] = S[2 + D + a];
    }
    const double m2 = S[1 + D];
    int o = 2 + 2 * D;
    for (int a = 0; a < D; ++a)
        for (int b = a; b < D; ++b) {
            M[a][b] = M[b][a] = S[o];
            ++o;
        }
    double del[3] = {0, 0, 0}, mm = 0.0, dd = 0.0;
    for (int a = 0; a < 3; ++a) U[a] = Uref[a];
    for (int a = 0; a < D; ++a) {
        del[a] = m1[a] / m0;
        U[a] = Uref[a] + del[a];
        mm += m1[a] * m1[a];
        dd += del[a] * del[a];
    }
    rho = m0;
    T = (2.0 / 3.0) * (m2 - mm / m0) / m0;
    for (int a = 0; a < 3; ++a) q[a] = 0.0;
    for (int a = 0; a < D; ++a) {
        double Md = 0.0;
        for (int b = 0; b < D; ++b) Md += M[a][b] * del[b];
        q[a] = 0.5 * (m3[a] - 2.0 * Md - del[a] * m2 + 2.0 * dd * m1[a]);
    }
}

// f = (f* + r g^S)/(1 + r) over the nodes of fluid cell c, one wavefront;
// g^S from rho, U, T and the new heat flux q (the equilibrium of the update).
// Leaves the relaxed state's moment sums about U in S (every lane).
template <int D, typename T, typename DR>
__device__ void relax_cell(const DR &d, int cur, int c, double rho, const double U[3], double Tc, const double q[3],
                           double r, double *S)
{
    constexpr int PW = D == 2 ? kPartialWords2 : kPartialWords3;
    const int lane = threadIdx.x & 63;
    const double iT = 1.0 / Tc;
    const double A = (D == 2) ? rho / (kPi * Tc) : rho * pow(kPi * Tc, -1.5);
    const double coef = d.shk / (rho * Tc * Tc), c0 = 1.0 / (1.0 + r), halfT = 0.5 * Tc;
    double s[3];
    for (int a = 0; a < 3; ++a) s[a] = coef * q[a];
    T *f0 = (T *)d.f[cur][0] + (size_t)c * d.NV;
    T *f1 = D == 2 ? (T *)d.f[cur][1] + (size_t)c * d.NV : nullptr;
    double acc[PW];
#pragma unroll
    for (int j = 0; j < PW; ++j) acc[j] = 0.0;
    for (int k = lane; k < d.NV; k += 64) {
        double cc[3] = {0, 0, 0}, c2 = 0.0, cs = 0.0;
        for (int a = 0; a < D; ++a) {
            cc[a] = d.xi[a][k] - U[a];
            c2 += cc[a] * cc[a];
            cs += cc[a] * s[a];
        }
        const double a_ = c2 * iT, Ae = A * exp(-a_), w = d.w[k];
        const double r0 = fref<T>(d, 0, k);
        double n0, e;
        if (D == 2) {
            const double r1 = fref<T>(d, 1, k);
            const double g0 = Ae * (1.0 + cs * (2.0 * a_ - 4.0));
            const double g1 = halfT * Ae * (1.0 + cs * (2.0 * a_ - 2.0));
            const T t0 = (T)(((double)f0[k] + r0 + r * g0) * c0 - r0);
            const T t1 = (T)(((double)f1[k] + r1 + r * g1) * c0 - r1);
            f0[k] = t0;
            f1[k] = t1;
            n0 = (double)t0 + r0;
            e = c2 * n0 + ((double)t1 + r1);
        } else {
            const double g = Ae * (1.0 + cs * (2.0 * a_ - 5.0));
            const T t0 = (T)(((double)f0[k] + r0 + r * g) * c0 - r0);
            f0[k] = t0;
            n0 = (double)t0 + r0;
            e = c2 * n0;
        }
        acc[0] += w * n0;
        acc[1 + D] += w * e;
        int o = 2 + 2 * D;
        for (int a = 0; a < D; ++a) {
            acc[1 + a] += w * cc[a] * n0;
            acc[2 + D + a] += w * cc[a] * e;
            for (int b = a; b < D; ++b) acc[o++] += w * cc[a] * cc[b] * n0;
        }
    }
#pragma unroll
    for (int j = 0; j < PW; ++j) S[j] = wave_sum(acc[j]);
}

template <int D, typename TS, typename DR>
__device__ void fin_cells_relax(const DR &d, int cur, int slot, int blk)
{
    constexpr int PW = D == 2 ? kPartialWords2 : kPartialWords3;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double tmin = INFINITY;
    // convergence residual of Section 4, per conservative variable W = (rho,
    // rho U[3], rho E) with rho E = rho |U|^2 / 2 + 3 rho T / 4: the block's
    // sums of (W^{n+1} - W^n)^2 and of |W^{n+1}| (W^n: the parameters about
    // to be replaced)
    __shared__ double rsum[4][2 * kResVars];
    double rv[2 * kResVars];
#pragma unroll
    for (int i = 0; i < 2 * kResVars; ++i) rv[i] = 0.0;
    // one cell per wavefront: the cell's partial records are contiguous, lane
    // l sums word l % 16 of records l / 16, l / 16 + 4, ... in coalesced loads
    // the flag word, the cell record and the partial records are read
    // together (in bounds for every c < Nc), so the wavefront waits for
    // one round trip to memory instead of three
    const int c = blk * kFinCellsRelax + wv;
    const bool cin = c < d.Nc;
    const size_t cs = cin ? (size_t)c : 0;
    const int fl = d.cflag[cs];
    const double *cp = d.cellp + cs * kCellWords;
    const double Uref[3] = {cp[CW_U], cp[CW_U + 1], cp[CW_U + 2]};
    const double rho_old = cp[CW_RHO], T_old = cp[CW_T];
    const double *pp = d.part + cs * d.nchunk * kPartialStride;
    const int nw = d.nchunk * kPartialStride;
    // words lane, lane + 64, ... alternate between two sums (even rows to
    // acc, odd rows to acc2, in order); eight rows are loaded before they
    // are added, the last block with the rows past the end read as zero
    double acc = 0.0, acc2 = 0.0;
    int ow = lane;
    for (; ow + 7 * 64 < nw; ow += 8 * 64) {
        double v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = pp[ow + 64 * m];
#pragma unroll
        for (int m = 0; m < 8; m += 2) {
            acc += v[m];
            acc2 += v[m + 1];
        }
    }
    if (ow < nw) {
        double v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = ow + 64 * m < nw ? pp[ow + 64 * m] : 0.0;
#pragma unroll
        for (int m = 0; m < 8; m += 2) {
            acc += v[m];
            acc2 += v[m + 1];
        }
    }
    if (cin && !(fl & 1)) {
        acc += acc2;
        acc += __shfl_xor(acc, 16, 64);
        acc += __shfl_xor(acc, 32, 64);
        double S[PW];
#pragma unroll
        for (int j = 0; j < PW; ++j) S[j] = __shfl(acc, j, 64);
        double m0, U[3], T, q[3];
        moments_from_sums<D>(S, Uref, m0, U, T, q);
        // semi-implicit collision: the new heat flux in closed form, then
        // the backward-Euler relaxation of the cell's transported state and
        // the relaxed state's moments
        if (d.flags & kFlagImplicit) {
            const double r = d.ctrl->dt * (0.5 * m0 * T) / (d.mu0 * pow(T, d.omega));
            for (int a = 0; a < D; ++a) q[a] /= 1.0 + d.Pr * r;
            const double Us[3] = {U[0], U[1], U[2]};
            relax_cell<D, TS>(d, cur, c, m0, Us, T, q, r, S);
            moments_from_sums<D>(S, Us, m0, U, T, q);
        }
        const double Wo[kResVars] = {rho_old, rho_old * Uref[0], rho_old * Uref[1], rho_old * Uref[2],
                                     rho_old * (0.5 * (Uref[0] * Uref[0] + Uref[1] * Uref[1] + Uref[2] * Uref[2]) +
                                                0.75 * T_old)};
        const double Wn[kResVars] = {m0, m0 * U[0], m0 * U[1], m0 * U[2],
                                     m0 * (0.5 * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]) + 0.75 * T)};
#pragma unroll
        for (int i = 0; i < kResVars; ++i) {
            rv[i] = (Wn[i] - Wo[i]) * (Wn[i] - Wo[i]);
            rv[kResVars + i] = fabs(Wn[i]);
        }
        double tau = INFINITY;
        if (lane == 0) tau = write_cell(d, c, m0, U, T, q, D);
        tmin = fmin(tmin, tau);
    }
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 2 * kResVars; ++i) rsum[wv][i] = rv[i];
    __syncthreads();
    if (threadIdx.x < 2 * kResVars)
        d.respart[(size_t)blk * 2 * kResVars + threadIdx.x] =
            (rsum[0][threadIdx.x] + rsum[1][threadIdx.x]) + (rsum[2][threadIdx.x] + rsum[3][threadIdx.x]);
    tau_min_commit(d, slot, tmin);
}

template <int D, typename TS, typename DR>
__device__ void fin_cells_explicit(const DR &d, int cur, int slot, int blk)
{
    constexpr int PW = D == 2 ? kPartialWords2 : kPartialWords3;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane >> 4, l16 = lane & 15;
    // convergence residual of Section 4, per conservative variable W = (rho,
    // rho U[3], rho E) with rho E = rho |U|^2 / 2 + 3 rho T / 4: the block's
    // sums of (W^{n+1} - W^n)^2 and of |W^{n+1}| (W^n: the parameters about
    // to be replaced)
    __shared__ double rsum[4][2 * kResVars];
    double rv[2 * kResVars];
#pragma unroll
    for (int i = 0; i < 2 * kResVars; ++i) rv[i] = 0.0;
    // four cells per wavefront, 16 lanes each: lane l16 of a group sums word
    // l16 of the cell's partial records in record order (each load of the
    // group reads one contiguous 128-byte record); the flag word, the cell
    // record and the partial records are read together (in bounds for every
    // c < Nc), so the wavefront waits for one round trip to memory
    const int cw0 = blk * kFinCells + wv * 4;
    const int c = cw0 + grp;
    const bool cin = c < d.Nc;
    const size_t cs = cin ? (size_t)c : 0;
    const int fl = d.cflag[cs];
    const double *cp = d.cellp + cs * kCellWords;
    const double Uref[3] = {cp[CW_U], cp[CW_U + 1], cp[CW_U + 2]};
    const double rho_old = cp[CW_RHO], T_old = cp[CW_T];
    const double *pp = d.part + cs * d.nchunk * kPartialStride + l16;
    const int nr = d.nchunk;
    // the sums of the one-cell-per-wavefront finish in the same order, so
    // both instances give the same bits: records r = 4 t + g go to group g,
    // even t to e[g] and odd t to o[g], each in increasing t; then
    // (A0 + A1) + (A2 + A3) with A_g = e[g] + o[g].  Eight records (two t,
    // four g) are loaded before they are added; past the end they read as
    // zero.
    double e[4] = {0.0, 0.0, 0.0, 0.0}, o[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < nr; r += 8) {
        double v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = r + m < nr ? pp[(r + m) * kPartialStride] : 0.0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            e[g] += v[g];
            o[g] += v[4 + g];
        }
    }
    const double acc = ((e[0] + o[0]) + (e[1] + o[1])) + ((e[2] + o[2]) + (e[3] + o[3]));
    double S[PW];
#pragma unroll
    for (int j = 0; j < PW; ++j) S[j] = __shfl(acc, (lane & 48) + j, 64);
    const bool live = cin && !(fl & 1);
    double m0 = 1.0, U[3] = {0.0, 0.0, 0.0}, T = 1.0, q[3] = {0.0, 0.0, 0.0};
    if (live) moments_from_sums<D>(S, Uref, m0, U, T, q);
    double tau = INFINITY;
    if (live) {
        const double Wo[kResVars] = {rho_old, rho_old * Uref[0], rho_old * Uref[1], rho_old * Uref[2],
                                     rho_old * (0.5 * (Uref[0] * Uref[0] + Uref[1] * Uref[1] + Uref[2] * Uref[2]) +
                                                0.75 * T_old)};
        const double Wn[kResVars] = {m0, m0 * U[0], m0 * U[1], m0 * U[2],
                                     m0 * (0.5 * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]) + 0.75 * T)};
#pragma unroll
        for (int i = 0; i < kResVars; ++i) {
            rv[i] = (Wn[i] - Wo[i]) * (Wn[i] - Wo[i]);
            rv[kResVars + i] = fabs(Wn[i]);
        }
        if (l16 == 0) tau = write_cell(d, c, m0, U, T, q, D);
    }
    // the wavefront's residual sums over its four cells, in a fixed order
#pragma unroll
    for (int i = 0; i < 2 * kResVars; ++i) {
        double v = l16 == 0 ? rv[i] : 0.0;
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        rv[i] = v;
    }
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 2 * kResVars; ++i) rsum[wv][i] = rv[i];
    __syncthreads();
    if (threadIdx.x < 2 * kResVars)
        d.respart[(size_t)blk * 2 * kResVars + threadIdx.x] =
            (rsum[0][threadIdx.x] + rsum[1][threadIdx.x]) + (rsum[2][threadIdx.x] + rsum[3][threadIdx.x]);
    tau_min_commit(d, slot, tau);
}

// IMPL: the instance that can take the semi-implicit branch, one cell per
// wavefront (its relaxation pass uses the whole wavefront per cell and more
// than doubles the registers); the explicit instance finishes four cells
// per wavefront at about twice the occupancy.  The cells per workgroup of
// each instance (kFinCellsRelax, kFinCells) set the launch size and the
// residual partials' count on the host.
template <int D, typename TS, bool IMPL, typename DR>
__device__ __forceinline__ void fin_cells(const DR &d, int cur, int slot, int blk)
{
    if constexpr (IMPL)
        fin_cells_relax<D, TS>(d, cur, slot, blk);
    else
        fin_cells_explicit<D, TS>(d, cur, slot, blk);
}

template <int D, typename T, bool IMPL>
__global__ __launch_bounds__(256) void k_fill_fin(Dev d, int cur, int slot, int nfill, int dofin)
{
    if ((int)blockIdx.x < nfill) {
        const int nfc = fill_chunks(d);
        fill_incident<D, T>(d, cur, blockIdx.x / nfc, blockIdx.x % nfc);
        return;
    }
    if (dofin) fin_cells<D, T, IMPL>(d, cur, slot, blockIdx.x - nfill);
}

template <int D>
__global__ __launch_bounds__(256) void k_fill_specular(Dev d)
{
    const int nfc = fill_chunks(d);
    fill_specular<D>(d, blockIdx.x / nfc, blockIdx.x % nfc);
}

template <int D>
__global__ __launch_bounds__(256) void k_fill_ghost(Dev d)
{
    const int nfc = fill_chunks(d);
    fill_ghost<D>(d, blockIdx.x / nfc, blockIdx.x % nfc);
}

// workgroups are dispatched round-robin over the 8 XCDs; each XCD gets a
// contiguous run of tiles so that x-neighbouring tiles share its L2
__device__ __forceinline__ long long xcd_run(int nb) { return (long long)(blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3); }

// wavefront-uniform position of workgroup run index L in a batch: the solve
// s with blk0[s] <= L < blk0[s + 1]
__device__ __forceinline__ int batch_solve(const BatchArgs &a, long long L)
{
    int s = 0;
    while (s + 1 < a.n && L >= a.blk0[s + 1]) ++s;
    return s;
}
typedef const __attribute__((address_space(4))) Dev *cdev_p;

// the three fill phases over the (pair, chunk) workgroups of several solves
template <int D, typename T, bool IMPL>
__global__ __launch_bounds__(256) void k_fill_fin_batch(BatchArgs a)
{
    const int s = batch_solve(a, blockIdx.x);
    const auto &d = *(cdev_p)a.dev[s];
    const int b = blockIdx.x - (int)a.blk0[s];
    if (b < a.nfill[s]) {
        const int nfc = fill_chunks(d);
        fill_incident<D, T>(d, a.cur[s], b / nfc, b % nfc);
        return;
    }
    fin_cells<D, T, IMPL>(d, a.cur[s], a.slot[s], b - a.nfill[s]);
}

template <int D>
__global__ __launch_bounds__(256) void k_fill_specular_batch(BatchArgs a)
{
    const int s = batch_solve(a, blockIdx.x);
    const auto &d = *(cdev_p)a.dev[s];
    const int b = blockIdx.x - (int)a.blk0[s], nfc = fill_chunks(d);
    fill_specular<D>(d, b / nfc, b % nfc);
}

template <int D>
__global__ __launch_bounds__(256) void k_fill_ghost_batch(BatchArgs a)
{
    const int s = batch_solve(a, blockIdx.x);
    const auto &d = *(cdev_p)a.dev[s];
    const int b = blockIdx.x - (int)a.blk0[s], nfc = fill_chunks(d);
    fill_ghost<D>(d, b / nfc, b % nfc);
}

// direct two-pass moments of the current state (after create / set_state)
template <int D, typename T>
__global__ __launch_bounds__(256) void k_moments_direct(Dev d, int cur, int slot)
{
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    double tau = INFINITY;
    if (c < d.Nc && !(d.cflag[c] & 1)) {
        const T *f0 = (const T *)d.f[cur][0] + (size_t)c * d.NV;
        const T *f1 = D == 2 ? (const T *)d.f[cur][1] + (size_t)c * d.NV : nullptr;
        double rho = 0, m[3] = {0, 0, 0}, E2 = 0;
        for (int k = lane; k < d.NV; k += 64) {
            double h = (double)f0[k] + fref<T>(d, 0, k), x2 = 0.0;
            for (int a = 0; a < D; ++a) {
                double x = d.xi[a][k];
                x2 += x * x;
                m[a] += d.w[k] * x * h;
            }
            rho += d.w[k] * h;
            E2 += d.w[k] * (x2 * h + (D == 2 ? (double)f1[k] + fref<T>(d, 1, k) : 0.0));
        }
        rho = wave_sum(rho);
        E2 = wave_sum(E2);
        double U[3] = {0, 0, 0}, U2 = 0.0;
        for (int a = 0; a < D; ++a) {
            U[a] = wave_sum(m[a]) / rho;
            U2 += U[a] * U[a];
        }
        double Tc = 4.0 * (0.5 * E2 - 0.5 * rho * U2) / (3.0 * rho);
        double q[3] = {0, 0, 0};
        for (int k = lane; k < d.NV; k += 64) {
            double cc[3] = {0, 0, 0}, c2 = 0.0;
            for (int a = 0; a < D; ++a) {
                cc[a] = d.xi[a][k] - U[a];
                c2 += cc[a] * cc[a];
            }
            double E = c2 * ((double)f0[k] + fref<T>(d, 0, k)) + (D == 2 ? (double)f1[k] + fref<T>(d, 1, k) : 0.0);
            for (int a = 0; a < D; ++a) q[a] += d.w[k] * cc[a] * E;
        }
        for (int a = 0; a < D; ++a) q[a] = 0.5 * wave_sum(q[a]);
        if (lane == 0) tau = write_cell(d, c, rho, U, Tc, q, D);
    }
    tau_min_commit(d, slot, tau);
}

// ---------------------------------------------------------------- update

// ---------------------------------------------------------------- 2D update, marching in y
// Workgroup = TX wavefronts; wavefront w owns grid column i0 + w and its lanes
// own velocity nodes k0 + lane + 64 v (v < V).  The workgroup marches up a
// segment of rows.  Rows j-2..j+2 of the own column live in registers; row j
// of the TX columns plus two halo columns per side is exchanged through LDS,
// the x slopes of the TX + 2 cells the faces need are computed once per row
// (the two halo cells' by wavefronts 0..3, one array each) and shared
// through LDS, and the y slope of
// row j+1 and the flux state of face j+1/2 are carried to the next row.  Outer
// freestream ghosts are the freestream values (zero slope follows from the
// limiter); periodic ghosts wrap.  Solid face neighbours are replaced by the
// ghost value of the pair seen from the fluid cell, and faces toward a solid
// cell take the pair's ghost-side face value.

// cross-lane helpers on doubles (two 32-bit halves each)
__device__ __forceinline__ double mk_dbl(unsigned hi, unsigned lo)
{
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// v_permlane32_swap: the upper 32 lanes of x trade places with the lower 32
// lanes of y
__device__ __forceinline__ void swap32(double &x, double &y)
{
    unsigned long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
    auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bx, (unsigned)by, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
    x = mk_dbl(hi[0], lo[0]);
    y = mk_dbl(hi[1], lo[1]);
}

// v_permlane16_swap: within each 32-lane half, lanes 16..31 of x trade places
// with lanes 0..15 of y
__device__ __forceinline__ void swap16(double &x, double &y)
{
    unsigned long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
    auto lo = __builtin_amdgcn_permlane16_swap((unsigned)bx, (unsigned)by, false, false);
    auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
    x = mk_dbl(hi[0], lo[0]);
    y = mk_dbl(hi[1], lo[1]);
}

// DPP rotation within 16-lane rows
template <int CTRL>
__device__ __forceinline__ double dpp(double x)
{
    unsigned long long b = __double_as_longlong(x);
    unsigned lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, false);
    unsigned hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return mk_dbl(hi, lo);
}
constexpr int kRowRor1 = 0x121, kRowRor2 = 0x122, kRowRor4 = 0x124, kRowRor8 = 0x128;

// sums S[0..8] over the 64 lanes.  Three exchange steps halve the number of
// values each lane carries (after them lane l holds value 4 b5 + 2 b4 + b3
// summed over the 8 lanes that share bits 0..2), three rotate-and-add steps
// finish the sums in lanes 8m + 7 (whose sources stay inside their group).  On return lane 8m + 7 holds the total of
// S[m] for m < 8 and lanes 7 and 15 hold the total of S[8].
__device__ __forceinline__ void reduce9(const double S[9], double &r8, double &s8)
{
    const int lane = threadIdx.x & 63;
    double a[4], b[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double x = S[i], y = S[4 + i];
        swap32(x, y);
        a[i] = x + y;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        double x = a[i], y = a[2 + i];
        swap16(x, y);
        b[i] = x + y;
    }
    const bool b3 = lane & 8;
    double c = (b3 ? b[1] : b[0]) + dpp<kRowRor8>(b3 ? b[0] : b[1]);
    c += dpp<kRowRor4>(c);
    c += dpp<kRowRor2>(c);
    c += dpp<kRowRor1>(c);
    r8 = c;
    double s = S[8], t = S[8];
    swap32(s, t);
    s += t;
    t = s;
    swap16(s, t);
    s += t;
    s += dpp<kRowRor8>(s);
    s += dpp<kRowRor4>(s);
    s += dpp<kRowRor2>(s);
    s += dpp<kRowRor1>(s);
    s8 = s;
}

// sums S[0..15] over the 64 lanes with the exchange steps of reduce9 stopped
// one step earlier: afterwards lane l carries S[2 g + i] for i = 0, 1 and
// g = (l >> 3) & 7, summed over the lanes that share bits 3..5; three
// rotate-and-add steps finish both sums in lanes 8 g + 7 (out[0], out[1]).
__device__ __forceinline__ void reduce16(const double S[16], double out[2])
{
    const int lane = threadIdx.x & 63;
    double a[8], b[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        double x = S[i], y = S[8 + i];
        swap32(x, y);
        a[i] = x + y;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double x = a[i], y = a[4 + i];
        swap16(x, y);
        b[i] = x + y;
    }
    const bool b3 = lane & 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        double c = (b3 ? b[2 + i] : b[i]) + dpp<kRowRor8>(b3 ? b[i] : b[2 + i]);
        c += dpp<kRowRor4>(c);
        c += dpp<kRowRor2>(c);
        c += dpp<kRowRor1>(c);
        out[i] = c;
    }
}

// barrier for LDS traffic only: global loads issued before it stay in flight
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// wavefront-uniform values in scalar registers
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// read-only tables indexed by wavefront-uniform values go through the
// scalar cache (constant address space): the loads land in scalar registers
typedef const __attribute__((address_space(4))) int *cint_p;
typedef const __attribute__((address_space(4))) double *cdbl_p;

// ---------------------------------------------------------------- 2D update
//
// Raw buffer access: the descriptor carries the base address and the byte
// length of one velocity row, so the address arithmetic of a row is scalar,
// lanes past the end of the row read 0, and their stores are dropped.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t brsrc;
constexpr int kRsrcW3 = 0x00020000;  // descriptor word 3 on the gfx9 family: 32-bit data format
constexpr int kOob = 0x40000000;     // an offset past every buffer

__device__ __forceinline__ brsrc mk_rsrc(const void *p, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, kRsrcW3);
}
__device__ __forceinline__ double bld(brsrc r, int off, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float bld(brsrc r, int off, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void bst(brsrc r, int off, double x)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, off, 0, 0);
}
__device__ __forceinline__ void bst(brsrc r, int off, float x)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, off, 0, 0);
}

// half the van Leer limited slope of one-sided differences d1, d2:
// d1 d2 / (d1 + d2) when they have the same sign, else 0 (d1 d2 > 0 keeps
// |d1 + d2| far from the reciprocal's overflow range).  The hardware
// reciprocal (relative error below 5e-8) takes one Newton step, leaving a
// few units in the last place.
__device__ __forceinline__ double vl_half(double d1, double d2)
{
    const double p = d1 * d2, den = d1 + d2;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(fma(-den, r, 1.0), r, r);
    return p > 0.0 ? p * r : 0.0;
}
__device__ __forceinline__ float vl_half(float d1, float d2)
{
    const float p = d1 * d2, den = d1 + d2;
    return p > 0.0f ? p * __builtin_amdgcn_rcpf(den) : 0.0f;
}

// outgoing state f + sign(xi) h toward the downwind face: the sign bit of
// the node velocity is XORed into h instead of multiplying by a stored +-1
__device__ __forceinline__ double ostate(double h, double f, double xi)
{
    const unsigned long long s = __builtin_bit_cast(unsigned long long, xi) & 0x8000000000000000ull;
    return f + __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, h) ^ s);
}
__device__ __forceinline__ float ostate(float h, float f, double xi)
{
    const unsigned s = (unsigned)(__builtin_bit_cast(unsigned long long, xi) >> 32) & 0x80000000u;
    return f + __builtin_bit_cast(float, __builtin_bit_cast(unsigned, h) ^ s);
}

// exp(x) for x <= 0: x = (32 m + j) ln2/32 + r with |r| <= ln2/64, so
// exp(x) = 2^m 2^(j/32) exp(r); 2^(j/32) comes from a 32-entry table and
// exp(r) from its degree-6 Taylor polynomial (truncation below 4e-18
// relative).  Below -746 the result underflows to 0.
__device__ __forceinline__ double exp_neg(double x, const double *tab)
{
    constexpr double kInvL = 46.16624130844683;       // 32 / ln 2
    constexpr double kLhi = 0.02166084939249829;      // ln 2 / 32, leading part
    constexpr double kLlo = 7.247021293269686e-19;    // ln 2 / 32 - kLhi
    x = fmax(x, -746.0);
    const double n = __builtin_rint(x * kInvL);
    double r = fma(-n, kLhi, x);
    r = fma(-n, kLlo, r);
    double p = fma(r, 1.0 / 720, 1.0 / 120);
    p = fma(p, r, 1.0 / 24);
    p = fma(p, r, 1.0 / 6);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    const int ni = (int)n;
    return ldexp(tab[ni & 31] * p, ni >> 5);
}

// ghost value / ghost-side face value of the pair seen from fluid cell c in
// direction dir (2 axis + side), at byte offset k8 = 8 k of node k; OFF: as
// an offset from the freestream (the 2D FP32 storage)
template <typename T, bool OFF, typename DR>
__device__ __forceinline__ T ghost_at(const DR &d, int A, int c, int dir, int k8)
{
    const int p = ((cint_p)d.pnb)[6 * c + dir];
    const double g = bld(mk_rsrc(d.ghost[A] + (size_t)p * d.NV, d.NV * 8), k8, double());
    if constexpr (OFF)
        return (T)(g - bld(mk_rsrc(d.fr[A], d.NV * 8), k8, double()));
    else
        return (T)g;
}
template <typename T, bool OFF, typename DR>
__device__ __forceinline__ T facev_at(const DR &d, int A, int c, int dir, int k8)
{
    const int p = ((cint_p)d.pnb)[6 * c + dir];
    const double g = bld(mk_rsrc(d.face[A] + (size_t)p * d.NV, d.NV * 8), k8, double());
    if constexpr (OFF)
        return (T)(g - bld(mk_rsrc(d.fr[A], d.NV * 8), k8, double()));
    else
        return (T)g;
}

// One workgroup = TX wavefronts = TX adjacent columns i0..i0+TX-1, rows
// j0..j1-1, and one chunk of 64 V velocity nodes (lane l holds nodes
// chunk*64V + 64 v + l).  Each wavefront marches its column upward.  Per row
// j the row is staged in LDS with two halo columns per side, the outgoing
// x-face states (f + sigma/2 toward the downwind side) are exchanged through
// LDS, and the y direction is carried in registers: rows j..j+2 are held, row
// j+3 arrives one row ahead, and the outgoing y state of row j and the face
// j-1/2 come from the previous row.  The Shakhov relaxation and the forward
// Euler update follow, then the moments of the new state about U^n are summed
// across the wavefront into one partial record per (cell, chunk).
//
// Rows touching the immersed boundary (flag bits of rows j and j+1) take the
// near path with the pair ghost and face values; every other row runs a
// branch-free path whose only memory traffic is the prefetch, the stores, the
// partial record and the next row's cell record, so loads stay in flight.
template <typename T, int V, int TX, bool WALLS, typename DR>
__device__ __forceinline__ void update2d_tile(const DR &d, int cur, int slot, int LY, int ntx, int nys, int ncv, int L)
{
    constexpr int W = 64 * V;
    constexpr int ST = (int)sizeof(T);
    constexpr int NEARX = CF_SOLID | CF_XM | CF_XP;
    constexpr int NEARALL = CF_SOLID | CF_XM | CF_XP | CF_YM | CF_YP;
    __shared__ T fb[2][TX + 4][W];
    __shared__ T ob[2][TX + 2][W];
    __shared__ double etab[32];
    __shared__ int flw[TX];
    if (threadIdx.x < 32) etab[threadIdx.x] = exp2((double)threadIdx.x * (1.0 / 32));

    const double tmin = __longlong_as_double((long long)d.ctrl->tau_bits[slot]);
    const double dt = d.cfl / (d.adv + 1.0 / tmin);
    if (L == 0 && threadIdx.x == 0) {
        d.ctrl->tau_bits[slot ^ 1] = kInfBits;
        d.ctrl->dt = dt;
        d.ctrl->time += dt;
        d.ctrl->step += 1;
    }
    const int tx = L % ntx, ys = (L / ntx) % nys, ch = L / (ntx * nys);
    const int nx = d.n[0], ny = d.n[1], NV = d.NV;
    const int i0 = tx * TX, j0 = ys * LY, j1 = min(j0 + LY, ny);
    const int lane = threadIdx.x & 63;
    const int w = uni(threadIdx.x >> 6);
    const int i = i0 + w;
    const bool col_in = i < nx;
    // WALLS: the outer boundary is walls, diffuse or specular (a separate
    // instantiation, so the other boundaries keep their row addressing)
    const bool per = !WALLS && d.outer != 0;
    const int rowb = NV * ST;
    const size_t rstride = (size_t)nx * (size_t)rowb;

    const char *fsr[2] = {(const char *)d.fsT[0], (const char *)d.fsT[1]};
    // tile column -> grid column (periodic wrap); fs: the freestream row;
    // xw: side of the x wall whose ghost rows stand in for the column
    auto colmap = [&](int ic, bool &fs, int &xw) -> int {
        const bool out = ic < 0 || ic >= nx;
        fs = !WALLS && !per && out;
        xw = WALLS && out ? (ic < 0 ? -1 : 1) : 0;
        return ic < 0 ? ic + nx : (ic >= nx ? ic - nx : ic);
    };
    // velocity row of array A at row jr of a column whose row 0 starts at
    // col (grid column ic; fs: the column reads the freestream row; walls:
    // rows of an x-wall column are its ghost rows, rows beyond the grid in
    // y are the y-wall ghost rows of column ic; both ghost layers of a wall
    // hold the same row, so the ghost's slope is zero)
    auto rowp = [&](int A, const char *col, bool cfs, int xw, int ic, int jr) -> const char * {
        const bool in = jr >= 0 && jr < ny;
        if constexpr (WALLS) {
            if (xw) return col + (size_t)(unsigned)min(max(jr, 0), ny - 1) * rowb;
            if (!in) return (const char *)d.wallT[A] + (size_t)(unsigned)(2 * ny + (jr < 0 ? 0 : nx) + ic) * rowb;
            return col + (size_t)(unsigned)jr * rstride;
        } else {
            const int jw = jr < 0 ? jr + ny : (jr >= ny ? jr - ny : jr);
            const bool usefs = cfs || (!in && !per);
            return usefs ? fsr[A] : col + (size_t)(unsigned)jw * rstride;
        }
    };
    auto ldflag = [&](int ic, int jr) -> int {
        const bool in = ic >= 0 && ic < nx && jr >= 0 && jr < ny;
        return (int)__builtin_amdgcn_raw_buffer_load_b32(mk_rsrc(d.cflag + (in ? ic + nx * jr : 0), in ? 4 : 0), 0, 0, 0);
    };
    int koff[V];
    double xx[V], xy[V], wk[V];
    // FP32 storage: the stored values are offsets from the freestream (fref)
    constexpr bool SHIFT = sizeof(T) == 4;
    double rf0[V], rf1[V];
    // FP64 keeps fewer per-lane values, so its V = 2 form runs three
    // wavefronts per SIMD: the sign of the node velocity is XORed into the
    // half slope (ostate), |xi|/dx is formed where used, and the cell record
    // lives in scalar registers; FP32 keeps them in vector registers
    constexpr bool LEAN = sizeof(T) == 8;
    T axp[V], ayq[V], sx[V], sy[V];
    bool pos[V], py[V];
    const T idx = (T)d.inv_dx[0], idy = (T)d.inv_dx[1];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int k = ch * W + v * 64 + lane;
        const int kc = min(k, NV - 1);
        koff[v] = k * ST;
        xx[v] = d.xi[0][kc];
        xy[v] = d.xi[1][kc];
        wk[v] = k < NV ? d.w[kc] : 0.0;
        if constexpr (SHIFT) {
            rf0[v] = d.fr[0][kc];
            rf1[v] = d.fr[1][kc];
        }
        pos[v] = xx[v] > 0.0;
        py[v] = xy[v] > 0.0;
        if constexpr (!LEAN) {
            axp[v] = (T)fabs(xx[v]) * idx;
            ayq[v] = (T)xy[v] * idy;
            sx[v] = pos[v] ? T(1) : T(-1);
            sy[v] = py[v] ? T(1) : T(-1);
        }
    }
    // outgoing states toward the downwind x / y face
    auto ostx = [&](T h, T f, int v) -> T {
        if constexpr (LEAN)
            return ostate(h, f, xx[v]);
        else
            return fma(sx[v], h, f);
    };
    auto osty = [&](T h, T f, int v) -> T {
        if constexpr (LEAN)
            return ostate(h, f, xy[v]);
        else
            return fma(sy[v], h, f);
    };

    // cell record of (i, jr): parameters of the update and the flag word of
    // the cell above
    auto ldrec = [&](int jr, double (&P)[8], int &fup) {
        const bool in = col_in && jr < ny;
        const size_t cc = in ? (size_t)(i + nx * jr) : 0;
        if constexpr (LEAN) {
            const cdbl_p q = (cdbl_p)(d.cellq + cc * kQWords);
#pragma unroll
            for (int m = 0; m < 8; ++m) P[m] = q[m];
            fup = in ? ((cint_p)q)[16] : 0;
        } else {
            const brsrc r = mk_rsrc(d.cellq + cc * kQWords, in ? 8 * kQWords : 0);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(r, 16 * m, 0, 0);
                P[2 * m] = __builtin_bit_cast(double, u32x2{u.x, u.y});
                P[2 * m + 1] = __builtin_bit_cast(double, u32x2{u.z, u.w});
            }
            fup = (int)__builtin_amdgcn_raw_buffer_load_b32(r, 64, 0, 0);
        }
    };

    bool cfs;
    int cxw;
    const int ie = colmap(i, cfs, cxw);
    // halo columns staged by wavefronts 0..3
    const int hcol = w < 2 ? i0 - 2 + w : i0 + TX + (w - 2);
    const int hpos = w < 2 ? w : TX + 2 + (w - 2);
    const bool hload = w < 4;
    // outgoing x states of the two halo cells next to the tile, one (side,
    // array) unit per wavefront 0..3: side = w >> 1 (column i0 - 1 or
    // i0 + TX), array = w & 1; flags from the adjacent tile cell's word
    const bool hunit = w < 4;
    const bool hright = (w >> 1) & 1;
    const int hA = w & 1;
    const int spos = hright ? TX + 1 : 0;
    bool hfs;
    int hxw;
    const int he = colmap(hcol, hfs, hxw);
    const char *fcol[2], *hcolp[2];
    char *gcol[2];
#pragma unroll
    for (int A = 0; A < 2; ++A) {
        const char *wr = WALLS ? (const char *)d.wallT[A] : nullptr;
        fcol[A] = cxw ? wr + (size_t)(cxw < 0 ? 0 : ny) * rowb : (const char *)d.f[cur][A] + (size_t)ie * rowb;
        hcolp[A] = hxw ? wr + (size_t)(hxw < 0 ? 0 : ny) * rowb : (const char *)d.f[cur][A] + (size_t)he * rowb;
        gcol[A] = (char *)d.f[cur ^ 1][A] + (size_t)ie * rowb;
    }

    // rows in flight, selected modulo 4 by the unrolled row position
    T R[4][2][V];
    T OY[2][2][V], FD[2][2][V], HH[2][2][V];
    double P[8];
    int FL0, fup;
    {
        T fm2[2][V], fm1[2][V];
#pragma unroll
        for (int A = 0; A < 2; ++A) {
            const brsrc r0 = mk_rsrc(rowp(A, fcol[A], cfs, cxw, ie, j0 - 2), rowb);
            const brsrc r1 = mk_rsrc(rowp(A, fcol[A], cfs, cxw, ie, j0 - 1), rowb);
            const brsrc r2 = mk_rsrc(rowp(A, fcol[A], cfs, cxw, ie, j0), rowb);
            const brsrc r3 = mk_rsrc(rowp(A, fcol[A], cfs, cxw, ie, j0 + 1), rowb);
            const brsrc r4 = mk_rsrc(rowp(A, fcol[A], cfs, cxw, ie, j0 + 2), rowb);
            const brsrc rh = mk_rsrc(rowp(A, hcolp[A], hfs, hxw, he, j0), hload ? rowb : 0);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                fm2[A][v] = bld(r0, koff[v], T());
                fm1[A][v] = bld(r1, koff[v], T());
                R[0][A][v] = bld(r2, koff[v], T());
                R[1][A][v] = bld(r3, koff[v], T());
                R[2][A][v] = bld(r4, koff[v], T());
                HH[0][A][v] = bld(rh, koff[v], T());
            }
        }
        const int flm1 = uni(ldflag(i, j0 - 1));
        FL0 = uni(ldflag(i, j0));
        ldrec(j0, P, fup);
        const int c0 = i + nx * j0;
        // outgoing y states of rows j0-1 and j0, and the face j0-1/2
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                T fm = fm2[A][v], fp = R[0][A][v];
                if (flm1 & CF_YM) fm = ghost_at<T, SHIFT>(d, A, c0 - nx, 2, koff[v] * (8 / ST));
                if (flm1 & CF_YP) fp = ghost_at<T, SHIFT>(d, A, c0 - nx, 3, koff[v] * (8 / ST));
                const T hm = (flm1 & CF_SOLID) ? T(0) : vl_half(fm1[A][v] - fm, fp - fm1[A][v]);
                const T oym = osty(hm, fm1[A][v], v);
                fm = fm1[A][v];
                fp = R[1][A][v];
                if (FL0 & CF_YM) fm = ghost_at<T, SHIFT>(d, A, c0, 2, koff[v] * (8 / ST));
                if (FL0 & CF_YP) fp = ghost_at<T, SHIFT>(d, A, c0, 3, koff[v] * (8 / ST));
                const T h0 = (FL0 & CF_SOLID) ? T(0) : vl_half(R[0][A][v] - fm, fp - R[0][A][v]);
                OY[0][A][v] = osty(h0, R[0][A][v], v);
                T F;
                if (py[v])
                    F = !(flm1 & CF_SOLID) ? oym : ((FL0 & CF_SOLID) ? T(0) : facev_at<T, SHIFT>(d, A, c0, 2, koff[v] * (8 / ST)));
                else
                    F = !(FL0 & CF_SOLID) ? OY[0][A][v] : ((flm1 & CF_SOLID) ? T(0) : facev_at<T, SHIFT>(d, A, c0 - nx, 3, koff[v] * (8 / ST)));
                FD[0][A][v] = F;
            }
        __builtin_amdgcn_s_waitcnt(0);
    }

    int j = j0;
    auto row = [&](auto S_) {
        constexpr int S = decltype(S_)::value;
        T(&f0)[2][V] = R[S & 3];
        T(&f1)[2][V] = R[(S + 1) & 3];
        T(&f2)[2][V] = R[(S + 2) & 3];
        T(&f3)[2][V] = R[(S + 3) & 3];
        T(&oy0)[2][V] = OY[S & 1];
        T(&oy1)[2][V] = OY[(S + 1) & 1];
        T(&Fdn)[2][V] = FD[S & 1];
        T(&Fup)[2][V] = FD[(S + 1) & 1];
        T(&hcur)[2][V] = HH[S & 1];
        T(&hnext)[2][V] = HH[(S + 1) & 1];
        const int c = i + nx * j;

        // prefetch: own column row j+3, halo column row j+1.  The loads are
        // issued at a raised wavefront priority: the three wavefronts of a
        // SIMD compete for issue, and a wavefront that reaches its loads
        // then gets them in flight ahead of the others' arithmetic (the
        // FP64 update runs 1-2 % faster; the results do not change)
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int A = 0; A < 2; ++A) {
            const brsrc r3 = mk_rsrc(rowp(A, fcol[A], cfs, cxw, ie, j + 3), rowb);
            const brsrc rh = mk_rsrc(rowp(A, hcolp[A], hfs, hxw, he, j + 1), hload ? rowb : 0);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                f3[A][v] = bld(r3, koff[v], T());
                hnext[A][v] = bld(rh, koff[v], T());
            }
        }
        __builtin_amdgcn_s_setprio(0);

        // stage row j
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                fb[A][w + 2][v * 64 + lane] = f0[A][v];
                if (hload) fb[A][hpos][v * 64 + lane] = hcur[A][v];
            }
        if (lane == 0) flw[w] = FL0;
        lds_barrier();

        // outgoing x states of the own cell and of the halo cells
        T ox[2][V];
        auto xstate = [&](auto near_tag, int fl, int cc, int p0, T (&out)[2][V], bool keep) {
            constexpr bool NEAR = decltype(near_tag)::value;
#pragma unroll
            for (int A = 0; A < 2; ++A)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    T fm = fb[A][p0][v * 64 + lane];
                    const T fc = fb[A][p0 + 1][v * 64 + lane];
                    T fp = fb[A][p0 + 2][v * 64 + lane];
                    if (NEAR && (fl & CF_XM)) fm = ghost_at<T, SHIFT>(d, A, cc, 0, koff[v] * (8 / ST));
                    if (NEAR && (fl & CF_XP)) fp = ghost_at<T, SHIFT>(d, A, cc, 1, koff[v] * (8 / ST));
                    T h = vl_half(fc - fm, fp - fc);
                    if (NEAR && (fl & CF_SOLID)) h = T(0);
                    const T o = ostx(h, fc, v);
                    if (keep) out[A][v] = o;
                    ob[A][p0][v * 64 + lane] = o;
                }
            // the pair loads of the near path are complete here, so the
            // prefetch of the following rows is not waited for at the join
            if (NEAR) __builtin_amdgcn_s_waitcnt(0);
        };
        // rows next to the boundary are few: the branch hints let the
        // register allocator put its scalar spill reloads on the near paths
        // (same results; 2D update 2-6 % faster, 3D FP32 22 %)
        if (__builtin_expect((FL0 & NEARX) != 0, 0))
            xstate(std::true_type{}, FL0, c, w + 1, ox, true);
        else
            xstate(std::false_type{}, 0, c, w + 1, ox, true);
        if (hunit) {
            // flag word of the halo cell, from the adjacent tile cell's flags
            const int fa = uni(flw[hright ? TX - 1 : 0]);
            const int flh = hright ? (((fa & CF_XP) ? CF_SOLID : 0) | ((fa & CF_SOLID) ? CF_XM : 0) |
                                      ((fa & CF_XP2) ? CF_XP : 0))
                                   : (((fa & CF_XM) ? CF_SOLID : 0) | ((fa & CF_XM2) ? CF_XM : 0) |
                                      ((fa & CF_SOLID) ? CF_XP : 0));
            // grid index of the halo cell: the adjacent tile cell one step out
            const int ch_ = c + ((hright ? TX - 1 : 0) - w) + (hright ? 1 : -1);
            auto hstate = [&](auto near_tag) {
                constexpr bool NEAR = decltype(near_tag)::value;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    T fm = fb[hA][spos][v * 64 + lane];
                    const T fc = fb[hA][spos + 1][v * 64 + lane];
                    T fp = fb[hA][spos + 2][v * 64 + lane];
                    if (NEAR && (flh & CF_XM)) fm = ghost_at<T, SHIFT>(d, hA, ch_, 0, koff[v] * (8 / ST));
                    if (NEAR && (flh & CF_XP)) fp = ghost_at<T, SHIFT>(d, hA, ch_, 1, koff[v] * (8 / ST));
                    T h = vl_half(fc - fm, fp - fc);
                    if (NEAR && (flh & CF_SOLID)) h = T(0);
                    ob[hA][spos][v * 64 + lane] = ostx(h, fc, v);
                }
                if (NEAR) __builtin_amdgcn_s_waitcnt(0);
            };
            if (__builtin_expect(flh != 0, 0))
                hstate(std::true_type{});
            else
                hstate(std::false_type{});
        }
        lds_barrier();

        // y direction, fluxes, relaxation, update, moments
        const int FL1 = uni(fup);
        const bool upd = col_in && !(FL0 & CF_SOLID);
        const brsrc ws0 = mk_rsrc(gcol[0] + (size_t)(unsigned)j * rstride, col_in ? rowb : 0);
        const brsrc ws1 = mk_rsrc(gcol[1] + (size_t)(unsigned)j * rstride, col_in ? rowb : 0);
        const double U0 = P[0], U1 = P[1], invT = P[3], S0 = P[4], S1 = P[5];
        const double rate = dt * P[7];
        const double Ar = rate * P[2], ThAr = P[6] * Ar, c1 = 1.0 - rate;
        double m[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) m[q] = 0.0;
        auto body = [&](auto near_tag) {
            constexpr bool NEAR = decltype(near_tag)::value;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                T div[2];
#pragma unroll
                for (int A = 0; A < 2; ++A) {
                    T fm = f0[A][v], fp = f2[A][v];
                    if (NEAR && (FL1 & CF_YM)) fm = ghost_at<T, SHIFT>(d, A, c + nx, 2, koff[v] * (8 / ST));
                    if (NEAR && (FL1 & CF_YP)) fp = ghost_at<T, SHIFT>(d, A, c + nx, 3, koff[v] * (8 / ST));
                    T h1 = vl_half(f1[A][v] - fm, fp - f1[A][v]);
                    if (NEAR && (FL1 & CF_SOLID)) h1 = T(0);
                    oy1[A][v] = osty(h1, f1[A][v], v);
                    T F = py[v] ? oy0[A][v] : oy1[A][v];
                    if (NEAR) {
                        if (py[v]) {
                            if (FL0 & CF_SOLID) F = (FL1 & CF_SOLID) ? T(0) : facev_at<T, SHIFT>(d, A, c + nx, 2, koff[v] * (8 / ST));
                        } else {
                            if (FL1 & CF_SOLID) F = (FL0 & CF_SOLID) ? T(0) : facev_at<T, SHIFT>(d, A, c, 3, koff[v] * (8 / ST));
                        }
                    }
                    Fup[A][v] = F;
                    // the upwind neighbour's outgoing state is the face state on the upwind side
                    T nbs = ob[A][pos[v] ? w : w + 2][v * 64 + lane];
                    if (NEAR && pos[v] && (FL0 & CF_XM)) nbs = facev_at<T, SHIFT>(d, A, c, 0, koff[v] * (8 / ST));
                    if (NEAR && !pos[v] && (FL0 & CF_XP)) nbs = facev_at<T, SHIFT>(d, A, c, 1, koff[v] * (8 / ST));
                    const T ax = LEAN ? (T)fabs(xx[v]) * idx : axp[v], ay = LEAN ? (T)xy[v] * idy : ayq[v];
                    div[A] = fma(ax, ox[A][v] - nbs, ay * (F - Fdn[A][v]));
                }
                if (NEAR && !upd) {
                    // solid cells are not advanced; carry their value
                    bst(ws0, koff[v], f0[0][v]);
                    bst(ws1, koff[v], f0[1][v]);
                    continue;
                }
                const double cx = xx[v] - U0, cy = xy[v] - U1;
                const double c2 = fma(cy, cy, cx * cx), cs = fma(cy, S1, cx * S0);
                const double a = c2 * invT;
                const double e = exp_neg(-a, etab);
                const double t0 = fma(a, 2.0, -4.0);
                double g0 = (Ar * e) * fma(cs, t0, 1.0);
                double g1 = (ThAr * e) * fma(cs, t0 + 2.0, 1.0);
                if constexpr (SHIFT) {
                    // relax the offset toward g - fref
                    g0 = fma(-rate, rf0[v], g0);
                    g1 = fma(-rate, rf1[v], g1);
                }
                const T st0 = (T)fma(-dt, (double)div[0], fma(c1, (double)f0[0][v], g0));
                const T st1 = (T)fma(-dt, (double)div[1], fma(c1, (double)f0[1][v], g1));
                bst(ws0, koff[v], st0);
                bst(ws1, koff[v], st1);
                double n0 = (double)st0, n1 = (double)st1;
                if constexpr (SHIFT) {
                    n0 += rf0[v];
                    n1 += rf1[v];
                }
                const double wh = wk[v] * n0, wE = wk[v] * fma(c2, n0, n1);
                const double tx_ = cx * wh, ty_ = cy * wh;
                m[0] += wh;
                m[1] += tx_;
                m[2] += ty_;
                m[3] += wE;
                m[4] = fma(cx, wE, m[4]);
                m[5] = fma(cy, wE, m[5]);
                m[6] = fma(cx, tx_, m[6]);
                m[7] = fma(cy, tx_, m[7]);
                m[8] = fma(cy, ty_, m[8]);
            }
            if (NEAR) __builtin_amdgcn_s_waitcnt(0);
        };
        if (__builtin_expect(((FL0 | FL1) & NEARALL) != 0, 0))
            body(std::true_type{});
        else
            body(std::false_type{});
        // cell record of the next row
        ldrec(j + 1, P, fup);
        // partial record: m0, m1x, m1y, m2, m3x, m3y, Mxx, Mxy, Myy
        double r8, s8;
        reduce9(m, r8, s8);
        const brsrc rp = mk_rsrc(d.part + ((size_t)c * ncv + ch) * kPartialStride, upd ? 72 : 0);
        bst(rp, (lane & 7) == 7 ? (lane >> 3) * 8 : kOob, r8);
        bst(rp, lane == 15 ? 64 : kOob, s8);
        FL0 = FL1;
    };

    for (;;) {
        row(std::integral_constant<int, 0>{});
        if (++j >= j1) break;
        row(std::integral_constant<int, 1>{});
        if (++j >= j1) break;
        row(std::integral_constant<int, 2>{});
        if (++j >= j1) break;
        row(std::integral_constant<int, 3>{});
        if (++j >= j1) break;
    }
}

// Ghost rows of the diffuse outer walls (2D), one workgroup per boundary
// cell and wall: the wall model of Section 2.3 at a domain face.  Velocities
// leaving the wall carry the wall Maxwellian at (U_wall, T_w) scaled by the
// density that zeroes the normal mass flux through the face against the
// cell's own h on the velocities toward the wall; those and the tangential
// velocities keep the cell's value.  The incoming flux of the unit wall
// Maxwellian depends on the wall side only and comes from the host (wall_in);
// the outgoing flux of the cell is summed here in FP64; the rows are written
// in the storage type.
//
// Specular outer walls: velocities leaving the wall carry the cell's own
// value at the mirrored velocity (the normal component reversed: node index
// N - 1 - i along the wall's axis), the others the cell's value.
template <typename T>
__global__ __launch_bounds__(256) void k_wall_fill(Dev d, int cur)
{
    const int nx = d.n[0], ny = d.n[1], NV = d.NV;
    const int r = blockIdx.x;
    int a, sd, cell;
    if (r < 2 * ny) {
        const int j = r < ny ? r : r - ny;
        a = 0;
        sd = r < ny ? -1 : 1;
        cell = (sd < 0 ? 0 : nx - 1) + nx * j;
    } else {
        const int q = r - 2 * ny, i = q < nx ? q : q - nx;
        a = 1;
        sd = q < nx ? -1 : 1;
        cell = i + nx * (sd < 0 ? 0 : ny - 1);
    }
    const T *h = (const T *)d.f[cur][0] + (size_t)cell * NV;
    const T *b = (const T *)d.f[cur][1] + (size_t)cell * NV;
    T *g0 = (T *)d.wallT[0] + (size_t)r * NV;
    T *g1 = (T *)d.wallT[1] + (size_t)r * NV;
    if (d.outer == kOuterSpecular) {
        const int N0 = d.vn[0];
        for (int k = threadIdx.x; k < NV; k += 256) {
            const double xn = sd * d.xi[a][k];
            int ix = k % N0, iy = k / N0;
            if (a == 0)
                ix = N0 - 1 - ix;
            else
                iy = d.vn[1] - 1 - iy;
            const int km = xn < 0.0 ? ix + N0 * iy : k;
            // stored values are offsets from node k's freestream value in the 2D FP32 form
            g0[k] = km == k ? h[k] : (T)((double)h[km] + fref<T>(d, 0, km) - fref<T>(d, 0, k));
            g1[k] = km == k ? b[k] : (T)((double)b[km] + fref<T>(d, 1, km) - fref<T>(d, 1, k));
        }
        return;
    }
    const double Ux = (a == 1 && sd > 0) ? d.lid_u : 0.0;
    const double iTw = 1.0 / d.Tw;
    // e^{-c^2/T_w} of the wall Maxwellian at node k
    auto ew = [&](int k) {
        const double cx = d.xi[0][k] - Ux, cy = d.xi[1][k];
        return exp(-(cx * cx + cy * cy) * iTw);
    };
    double out = 0.0;
    for (int k = threadIdx.x; k < NV; k += 256) {
        const double xn = sd * d.xi[a][k];
        if (xn > 0.0) out += d.w[k] * xn * ((double)h[k] + fref<T>(d, 0, k));
    }
    out = block_sum(out);
    // wall_in sums e^{-c^2/T_w} without the prefactor A_w, so out / wall_in
    // is rho_w A_w: the factor of e^{-c^2/T_w} in the ghost
    const double rA = out / d.wall_in[2 * a + (sd > 0 ? 1 : 0)];
    for (int k = threadIdx.x; k < NV; k += 256) {
        const double xn = sd * d.xi[a][k];
        if (xn < 0.0) {
            const double hv = rA * ew(k);
            g0[k] = (T)(hv - fref<T>(d, 0, k));
            g1[k] = (T)(0.5 * d.Tw * hv - fref<T>(d, 1, k));
        } else {
            g0[k] = h[k];
            g1[k] = b[k];
        }
    }
}

template <typename T, int V, int TX, bool WALLS>
__global__ __launch_bounds__(TX * 64) __attribute__((amdgpu_waves_per_eu(V == 1 ? 4 : 3)))
void k_update2d(Dev d, int cur, int slot, int LY, int ntx, int nys, int ncv)
{
    const long long L = xcd_run(gridDim.x);
    if (L >= (long long)ntx * nys * ncv) return;
    update2d_tile<T, V, TX, WALLS>(d, cur, slot, LY, ntx, nys, ncv, (int)L);
}

// one launch over the tiles of several solves (serving form): the solves'
// parameter blocks live in their workspaces, the per-solve launch values in
// the argument block
template <typename T, int V, int TX, bool WALLS>
__global__ __launch_bounds__(TX * 64) __attribute__((amdgpu_waves_per_eu(V == 1 ? 4 : 3)))
void k_update2d_batch(BatchArgs a)
{
    const long long L = xcd_run(gridDim.x);
    if (L >= a.blk0[a.n]) return;
    const int s = batch_solve(a, L);
    const auto &d = *(cdev_p)a.dev[s];
    update2d_tile<T, V, TX, WALLS>(d, a.cur[s], a.slot[s], a.LY[s], a.ntx[s], a.nys[s], a.ncv[s], (int)(L - a.blk0[s]));
}

// ---------------------------------------------------------------- 3D update, marching in z
//
// One workgroup = 16 wavefronts on a 4 x 4 tile of grid columns (i0 + tx,
// j0 + ty), a segment of planes k0..k1-1 and one chunk of 64 V velocity
// nodes.  Each wavefront marches its column in z: planes k..k+2 of the own
// column are held in registers and plane k+3 arrives one plane ahead, so the
// z slope of plane k+1 and the flux state of face k+1/2 are carried to the
// next plane as in the 2D update.  Plane k of the tile and of the two halo
// cells on each side along x and y (the cross-shaped stencil) is staged in
// LDS; each wavefront forms the outgoing x and y states of its own cell and
// the outgoing state of one of the 16 halo cells next to the tile (their
// flags follow from those of the adjacent tile cell), and the faces take the
// upwind neighbour's state from LDS.  Immersed-boundary substitutions are
// those of the 2D update with the z pair directions 4 and 5 added.
constexpr int kT3 = 4;  // tile edge along x

// staged plane of a 4 x TY tile: slot of tile position (x, y), x in [-2, 6),
// y in [-2, TY + 2), on the cross (rows 0..TY-1 with two halo columns per
// side: 8 slots each; then the two halo rows below and above, 4 slots each)
template <int TY>
__device__ __forceinline__ int xslot(int x, int y)
{
    return (y >= 0 && y < TY) ? y * (kT3 + 4) + x + 2 : TY * (kT3 + 4) + (y < 0 ? y + 2 : y - TY + 2) * kT3 + x;
}

template <typename T, int V, int TY>
__global__ __launch_bounds__(64 * kT3 * TY) __attribute__((amdgpu_waves_per_eu(TY == 4 || V == 1 ? 4 : 2)))
void k_update3d(Dev d, int cur, int slot, int LZ, int ntx, int nty, int nzs, int ncv)
{
    constexpr int NW = kT3 * TY;                    // wavefronts
    constexpr int NHL = kT3 * TY + 4 * kT3;         // halo cells staged per plane
    constexpr int NQ = (NHL + NW - 1) / NW;         // ... per wavefront
    constexpr int NHO = 2 * TY + 2 * kT3;           // halo cells whose outgoing state is formed
    constexpr int NO = (NHO + NW - 1) / NW;         // ... per wavefront
    constexpr int W = 64 * V;
    constexpr int ST = (int)sizeof(T);
    constexpr int NEAROWN = CF_SOLID | CF_XM | CF_XP | CF_YM | CF_YP;
    constexpr int NEARALL = NEAROWN | CF_ZM | CF_ZP;
    __shared__ T fb[TY * (kT3 + 4) + 4 * kT3][W];
    __shared__ T obx[TY][kT3 + 2][W];  // outgoing x states, x in [-1, 4]
    __shared__ T oby[TY + 2][kT3][W];  // outgoing y states, y in [-1, TY]
    __shared__ int flw[NW];
    __shared__ double etab[32];
    if (threadIdx.x < 32) etab[threadIdx.x] = exp2((double)threadIdx.x * (1.0 / 32));

    const double tmin = __longlong_as_double((long long)d.ctrl->tau_bits[slot]);
    const double dt = d.cfl / (d.adv + 1.0 / tmin);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.ctrl->tau_bits[slot ^ 1] = kInfBits;
        d.ctrl->dt = dt;
        d.ctrl->time += dt;
        d.ctrl->step += 1;
    }
    // contiguous runs of tiles per XCD (workgroups go round-robin over the 8)
    const int nb = gridDim.x;
    const int L = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    if (L >= ntx * nty * nzs * ncv) return;
    // tiles go out in stripes of 4 tile rows, x slowest within a stripe: the
    // 32 workgroups an XCD runs at once cover an 8 x 4 block of tiles whose
    // shared halo cells they load from its L2 at about the same plane
    const int Lt = L % (ntx * nty), zs = (L / (ntx * nty)) % nzs, ch = L / (ntx * nty * nzs);
    const int stripe = Lt / (4 * ntx), rows = min(4, nty - 4 * stripe), q = Lt - stripe * 4 * ntx;
    const int tX = q / rows, tY = 4 * stripe + q % rows;
    const int nx = d.n[0], ny = d.n[1], nz = d.n[2], NV = d.NV;
    const int i0 = tX * kT3, j0 = tY * TY, k0 = zs * LZ, k1 = min(k0 + LZ, nz);
    const int lane = threadIdx.x & 63;
    const int w = uni(threadIdx.x >> 6);
    const int tx = w & 3, ty = w >> 2;
    const int i = i0 + tx, j = j0 + ty;
    const bool col_in = i < nx && j < ny;
    const bool per = d.outer != 0;
    const int rowb = NV * ST;
    const size_t nxy = (size_t)nx * ny;
    const size_t pstride = nxy * (size_t)rowb;

    // first velocity row of grid column (ic, jc); fs: outside the grid and
    // not periodic, so the column reads the freestream row
    auto column = [&](int ic, int jc, bool &fs) -> size_t {
        fs = !per && (ic < 0 || ic >= nx || jc < 0 || jc >= ny);
        ic = ic < 0 ? ic + nx : (ic >= nx ? ic - nx : ic);
        jc = jc < 0 ? jc + ny : (jc >= ny ? jc - ny : jc);
        return ((size_t)ic + (size_t)nx * jc) * rowb;
    };
    auto planep = [&](const char *base, size_t col, bool cfs, const char *fsr, int kr) -> const char * {
        const bool in = kr >= 0 && kr < nz;
        const int kw = kr < 0 ? kr + nz : (kr >= nz ? kr - nz : kr);
        return (cfs || (!in && !per)) ? fsr : base + col + (size_t)(unsigned)kw * pstride;
    };
    auto ldflag = [&](int kr) -> int {
        const bool in = col_in && kr >= 0 && kr < nz;
        return (int)__builtin_amdgcn_raw_buffer_load_b32(
            mk_rsrc(d.cflag + (in ? (size_t)i + (size_t)nx * j + nxy * kr : 0), in ? 4 : 0), 0, 0, 0);
    };
    int koff[V];
    double xv[3][V], wk[V];
    bool pos[3][V];

    const T idx = (T)d.inv_dx[0], idy = (T)d.inv_dx[1], idz = (T)d.inv_dx[2];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int k = ch * W + v * 64 + lane;
        const int kc = min(k, NV - 1);
        koff[v] = k * ST;
        wk[v] = k < NV ? d.w[kc] : 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xv[a][v] = d.xi[a][kc];
            pos[a][v] = xv[a][v] > 0.0;
        }
    }

    // cell record of (i, j, kr): update parameters and the flag word of the
    // cell above
    auto ldrec = [&](int kr, double (&P)[9], int &fup) {
        // wavefront-uniform: scalar loads into scalar registers
        const bool in = col_in && kr < nz;
        const size_t cc = in ? (size_t)i + (size_t)nx * j + nxy * kr : 0;
        const cdbl_p q = (cdbl_p)(d.cellq + cc * kQWords);
#pragma unroll
        for (int m = 0; m < 9; ++m) P[m] = q[m];
        fup = in ? ((cint_p)q)[18] : 0;
    };

    const char *fcur = (const char *)d.f[cur][0];
    const char *fsr = (const char *)d.fsT[0];
    char *fnext = (char *)d.f[cur ^ 1][0];
    bool cfs;
    const size_t ccol = column(i, j, cfs);
    // halo cells staged by this wavefront: items w, w + NW, ... of the list
    // of x halo cells (columns -2, -1, 4, 5 of each tile row) followed by the
    // y halo cells (rows -2, -1, TY, TY + 1 of each tile column)
    size_t hcol[NQ];
    bool hfs[NQ], hon[NQ];
    int hsl[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int h = w + q * NW;
        hon[q] = h < NHL;
        int x, y;
        if (h < kT3 * TY) {
            x = (h & 3) < 2 ? (h & 3) - 2 : (h & 3) + 2;
            y = h >> 2;
        } else {
            const int h2 = min(h, NHL - 1) - kT3 * TY;
            x = h2 & 3;
            y = (h2 >> 2) < 2 ? (h2 >> 2) - 2 : TY + (h2 >> 2) - 2;
        }
        hcol[q] = column(i0 + x, j0 + y, hfs[q]);
        hsl[q] = xslot<TY>(x, y);
    }
    const int sown = xslot<TY>(tx, ty);

    T R[4][V], OZ[2][V], FD[2][V], HH[2][NQ][V];
    double P[9];
    int FL0, fup;
    {
        T fm2[V], fm1[V];
        const brsrc r0 = mk_rsrc(planep(fcur, ccol, cfs, fsr, k0 - 2), rowb);
        const brsrc r1 = mk_rsrc(planep(fcur, ccol, cfs, fsr, k0 - 1), rowb);
        const brsrc r2 = mk_rsrc(planep(fcur, ccol, cfs, fsr, k0), rowb);
        const brsrc r3 = mk_rsrc(planep(fcur, ccol, cfs, fsr, k0 + 1), rowb);
        const brsrc r4 = mk_rsrc(planep(fcur, ccol, cfs, fsr, k0 + 2), rowb);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            fm2[v] = bld(r0, koff[v], T());
            fm1[v] = bld(r1, koff[v], T());
            R[0][v] = bld(r2, koff[v], T());
            R[1][v] = bld(r3, koff[v], T());
            R[2][v] = bld(r4, koff[v], T());
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const brsrc rh = mk_rsrc(planep(fcur, hcol[q], hfs[q], fsr, k0), hon[q] ? rowb : 0);
#pragma unroll
            for (int v = 0; v < V; ++v) HH[0][q][v] = bld(rh, koff[v], T());
        }
        const int flm1 = uni(ldflag(k0 - 1));
        FL0 = uni(ldflag(k0));
        ldrec(k0, P, fup);
        const int c0 = (int)((size_t)i + (size_t)nx * j + nxy * k0);
        const int cm = c0 - (int)nxy;
        // outgoing z states of planes k0-1 and k0, and the face k0-1/2
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int k8 = koff[v] * (8 / ST);
            T fm = fm2[v], fp = R[0][v];
            if (flm1 & CF_ZM) fm = ghost_at<T, false>(d, 0, cm, 4, k8);
            if (flm1 & CF_ZP) fp = ghost_at<T, false>(d, 0, cm, 5, k8);
            const T hm = (flm1 & CF_SOLID) ? T(0) : vl_half(fm1[v] - fm, fp - fm1[v]);
            const T ozm = ostate(hm, fm1[v], xv[2][v]);
            fm = fm1[v];
            fp = R[1][v];
            if (FL0 & CF_ZM) fm = ghost_at<T, false>(d, 0, c0, 4, k8);
            if (FL0 & CF_ZP) fp = ghost_at<T, false>(d, 0, c0, 5, k8);
            const T h0 = (FL0 & CF_SOLID) ? T(0) : vl_half(R[0][v] - fm, fp - R[0][v]);
            OZ[0][v] = ostate(h0, R[0][v], xv[2][v]);
            T F;
            if (pos[2][v])
                F = !(flm1 & CF_SOLID) ? ozm : ((FL0 & CF_SOLID) ? T(0) : facev_at<T, false>(d, 0, c0, 4, k8));
            else
                F = !(FL0 & CF_SOLID) ? OZ[0][v] : ((flm1 & CF_SOLID) ? T(0) : facev_at<T, false>(d, 0, cm, 5, k8));
            FD[0][v] = F;
        }
        __builtin_amdgcn_s_waitcnt(0);
    }

    int k = k0;
    auto plane = [&](auto S_) {
        constexpr int S = decltype(S_)::value;
        T(&f0)[V] = R[S & 3];
        T(&f1)[V] = R[(S + 1) & 3];
        T(&f2)[V] = R[(S + 2) & 3];
        T(&f3)[V] = R[(S + 3) & 3];
        T(&oz0)[V] = OZ[S & 1];
        T(&oz1)[V] = OZ[(S + 1) & 1];
        T(&Fdn)[V] = FD[S & 1];
        T(&Fup)[V] = FD[(S + 1) & 1];
        T(&hc)[NQ][V] = HH[S & 1];
        T(&hn)[NQ][V] = HH[(S + 1) & 1];
        const int c = (int)((size_t)i + (size_t)nx * j + nxy * k);

        // prefetch: own column plane k+3, halo cells plane k+1
        {
            const brsrc r3 = mk_rsrc(planep(fcur, ccol, cfs, fsr, k + 3), rowb);
#pragma unroll
            for (int v = 0; v < V; ++v) f3[v] = bld(r3, koff[v], T());
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const brsrc rh = mk_rsrc(planep(fcur, hcol[q], hfs[q], fsr, k + 1), hon[q] ? rowb : 0);
#pragma unroll
                for (int v = 0; v < V; ++v) hn[q][v] = bld(rh, koff[v], T());
            }
        }
        // stage plane k
#pragma unroll
        for (int v = 0; v < V; ++v) fb[sown][v * 64 + lane] = f0[v];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (hon[q])
#pragma unroll
                for (int v = 0; v < V; ++v) fb[hsl[q]][v * 64 + lane] = hc[q][v];
        if (lane == 0) flw[w] = FL0;
        lds_barrier();

        // outgoing x and y states of the own cell
        T ox[V], oy[V];
        auto own = [&](auto near_tag) {
            constexpr bool NEAR = decltype(near_tag)::value;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int k8 = koff[v] * (8 / ST);
                const T fc = f0[v];
                T fm = fb[sown - 1][v * 64 + lane], fp = fb[sown + 1][v * 64 + lane];
                if (NEAR && (FL0 & CF_XM)) fm = ghost_at<T, false>(d, 0, c, 0, k8);
                if (NEAR && (FL0 & CF_XP)) fp = ghost_at<T, false>(d, 0, c, 1, k8);
                T h = vl_half(fc - fm, fp - fc);
                if (NEAR && (FL0 & CF_SOLID)) h = T(0);
                ox[v] = ostate(h, fc, xv[0][v]);
                obx[ty][tx + 1][v * 64 + lane] = ox[v];
                fm = fb[xslot<TY>(tx, ty - 1)][v * 64 + lane];
                fp = fb[xslot<TY>(tx, ty + 1)][v * 64 + lane];
                if (NEAR && (FL0 & CF_YM)) fm = ghost_at<T, false>(d, 0, c, 2, k8);
                if (NEAR && (FL0 & CF_YP)) fp = ghost_at<T, false>(d, 0, c, 3, k8);
                h = vl_half(fc - fm, fp - fc);
                if (NEAR && (FL0 & CF_SOLID)) h = T(0);
                oy[v] = ostate(h, fc, xv[1][v]);
                oby[ty + 1][tx][v * 64 + lane] = oy[v];
            }
            if (NEAR) __builtin_amdgcn_s_waitcnt(0);
        };
        if (FL0 & NEAROWN)
            own(std::true_type{});
        else
            own(std::false_type{});
        // outgoing states of the halo cells next to the tile (items w, w + NW,
        // ... of: x = -1 and x = 4 for each tile row, y = -1 and y = TY for
        // each tile column), with flags from the adjacent tile cell
#pragma unroll
        for (int q = 0; q < NO; ++q) {
            const int h = w + q * NW;
            if (h >= NHO) break;
            const bool hox = h < 2 * TY;
            const bool hside = hox ? h >= TY : h >= 2 * TY + kT3;
            const int hq = hox ? (hside ? h - TY : h) : (hside ? h - 2 * TY - kT3 : h - 2 * TY);
            const int hx = hox ? (hside ? kT3 : -1) : hq, hy = hox ? hq : (hside ? TY : -1);
            const int ax_ = hox ? (hside ? kT3 - 1 : 0) : hq, ay_ = hox ? hq : (hside ? TY - 1 : 0);
            const int fa = uni(flw[ay_ * kT3 + ax_]);
            int flh;
            if (hox)
                flh = hside ? (((fa & CF_XP) ? CF_SOLID : 0) | ((fa & CF_SOLID) ? CF_XM : 0) | ((fa & CF_XP2) ? CF_XP : 0))
                            : (((fa & CF_XM) ? CF_SOLID : 0) | ((fa & CF_XM2) ? CF_XM : 0) | ((fa & CF_SOLID) ? CF_XP : 0));
            else
                flh = hside ? (((fa & CF_YP) ? CF_SOLID : 0) | ((fa & CF_SOLID) ? CF_YM : 0) | ((fa & CF_YP2) ? CF_YP : 0))
                            : (((fa & CF_YM) ? CF_SOLID : 0) | ((fa & CF_YM2) ? CF_YM : 0) | ((fa & CF_SOLID) ? CF_YP : 0));
            const int sm = hox ? xslot<TY>(hx - 1, hy) : xslot<TY>(hx, hy - 1);
            const int sc = xslot<TY>(hx, hy);
            const int sp = hox ? xslot<TY>(hx + 1, hy) : xslot<TY>(hx, hy + 1);
            T *dst = hox ? &obx[hy][hx + 1][0] : &oby[hy + 1][hx][0];
            const int dm = hox ? 0 : 2;
            auto halo = [&](auto near_tag) {
                constexpr bool NEAR = decltype(near_tag)::value;
                // grid index of the halo cell: the adjacent tile cell one step out
                const int ch_ = c + (ax_ - tx) + (ay_ - ty) * nx + (hox ? (hside ? 1 : -1) : (hside ? nx : -nx));
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int k8 = koff[v] * (8 / ST);
                    T fm = fb[sm][v * 64 + lane];
                    const T fc = fb[sc][v * 64 + lane];
                    T fp = fb[sp][v * 64 + lane];
                    if (NEAR && (flh & (CF_XM | CF_YM))) fm = ghost_at<T, false>(d, 0, ch_, dm, k8);
                    if (NEAR && (flh & (CF_XP | CF_YP))) fp = ghost_at<T, false>(d, 0, ch_, dm + 1, k8);
                    T h = vl_half(fc - fm, fp - fc);
                    if (NEAR && (flh & CF_SOLID)) h = T(0);
                    dst[v * 64 + lane] = ostate(h, fc, hox ? xv[0][v] : xv[1][v]);
                }
                if (NEAR) __builtin_amdgcn_s_waitcnt(0);
            };
            if (__builtin_expect(flh != 0, 0))
                halo(std::true_type{});
            else
                halo(std::false_type{});
        }
        lds_barrier();

        // z direction, fluxes, relaxation, update, moments
        const int FL1 = uni(fup);
        const bool upd = col_in && !(FL0 & CF_SOLID);
        const int c1 = c + (int)nxy;
        const brsrc ws = mk_rsrc(fnext + ccol + (size_t)(unsigned)k * pstride, col_in ? rowb : 0);
        const double U0 = P[0], U1 = P[1], U2 = P[2], invT = P[4], S0 = P[5], S1 = P[6], S2 = P[7];
        const double rate = dt * P[8];
        const double Ar = rate * P[3], c1r = 1.0 - rate;
        double m[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) m[q] = 0.0;
        auto body = [&](auto near_tag) {
            constexpr bool NEAR = decltype(near_tag)::value;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int k8 = koff[v] * (8 / ST);
                T fm = f0[v], fp = f2[v];
                if (NEAR && (FL1 & CF_ZM)) fm = ghost_at<T, false>(d, 0, c1, 4, k8);
                if (NEAR && (FL1 & CF_ZP)) fp = ghost_at<T, false>(d, 0, c1, 5, k8);
                T h1 = vl_half(f1[v] - fm, fp - f1[v]);
                if (NEAR && (FL1 & CF_SOLID)) h1 = T(0);
                oz1[v] = ostate(h1, f1[v], xv[2][v]);
                T F = pos[2][v] ? oz0[v] : oz1[v];
                if (NEAR) {
                    if (pos[2][v]) {
                        if (FL0 & CF_SOLID) F = (FL1 & CF_SOLID) ? T(0) : facev_at<T, false>(d, 0, c1, 4, k8);
                    } else {
                        if (FL1 & CF_SOLID) F = (FL0 & CF_SOLID) ? T(0) : facev_at<T, false>(d, 0, c, 5, k8);
                    }
                }
                Fup[v] = F;
                // upwind neighbours' outgoing states are the face states on the upwind side
                T nx_ = obx[ty][pos[0][v] ? tx : tx + 2][v * 64 + lane];
                T ny_ = oby[pos[1][v] ? ty : ty + 2][tx][v * 64 + lane];
                if (NEAR && pos[0][v] && (FL0 & CF_XM)) nx_ = facev_at<T, false>(d, 0, c, 0, k8);
                if (NEAR && !pos[0][v] && (FL0 & CF_XP)) nx_ = facev_at<T, false>(d, 0, c, 1, k8);
                if (NEAR && pos[1][v] && (FL0 & CF_YM)) ny_ = facev_at<T, false>(d, 0, c, 2, k8);
                if (NEAR && !pos[1][v] && (FL0 & CF_YP)) ny_ = facev_at<T, false>(d, 0, c, 3, k8);
                const T ax = (T)fabs(xv[0][v]) * idx, ay = (T)fabs(xv[1][v]) * idy, az = (T)xv[2][v] * idz;
                const T div = fma(ax, ox[v] - nx_, fma(ay, oy[v] - ny_, az * (F - Fdn[v])));
                if (NEAR && !upd) {
                    // solid cells are not advanced; carry their value
                    bst(ws, koff[v], f0[v]);
                    continue;
                }
                const double cx = xv[0][v] - U0, cy = xv[1][v] - U1, cz = xv[2][v] - U2;
                const double c2 = fma(cz, cz, fma(cy, cy, cx * cx)), cs = fma(cz, S2, fma(cy, S1, cx * S0));
                const double a = c2 * invT;
                const double e = exp_neg(-a, etab);
                const double g = (Ar * e) * fma(cs, fma(a, 2.0, -5.0), 1.0);
                const T st = (T)fma(-dt, (double)div, fma(c1r, (double)f0[v], g));
                bst(ws, koff[v], st);
                const double n0 = (double)st;
                const double wh = wk[v] * n0, wE = c2 * wh;
                const double tx_ = cx * wh, ty_ = cy * wh, tz_ = cz * wh;
                m[0] += wh;
                m[1] += tx_;
                m[2] += ty_;
                m[3] += tz_;
                m[4] += wE;
                m[5] = fma(cx, wE, m[5]);
                m[6] = fma(cy, wE, m[6]);
                m[7] = fma(cz, wE, m[7]);
                m[8] = fma(cx, tx_, m[8]);
                m[9] = fma(cy, tx_, m[9]);
                m[10] = fma(cz, tx_, m[10]);
                m[11] = fma(cy, ty_, m[11]);
                m[12] = fma(cz, ty_, m[12]);
                m[13] = fma(cz, tz_, m[13]);
            }
            if (NEAR) __builtin_amdgcn_s_waitcnt(0);
        };
        if (__builtin_expect(((FL0 | FL1) & NEARALL) != 0, 0))
            body(std::true_type{});
        else
            body(std::false_type{});
        // cell record of the next plane
        ldrec(k + 1, P, fup);
        // partial record: m0, m1[3], m2, m3[3], M2 (xx, xy, xz, yy, yz, zz)
        double r[2];
        reduce16(m, r);
        const brsrc rp = mk_rsrc(d.part + ((size_t)c * ncv + ch) * kPartialStride, upd ? 8 * kPartialWords3 : 0);
        const u32x2 lo = __builtin_bit_cast(u32x2, r[0]), hi = __builtin_bit_cast(u32x2, r[1]);
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{lo.x, lo.y, hi.x, hi.y}, rp, (lane & 7) == 7 ? (lane >> 3) * 16 : kOob, 0, 0);
        FL0 = FL1;
    };

    for (;;) {
        plane(std::integral_constant<int, 0>{});
        if (++k >= k1) break;
        plane(std::integral_constant<int, 1>{});
        if (++k >= k1) break;
        plane(std::integral_constant<int, 2>{});
        if (++k >= k1) break;
        plane(std::integral_constant<int, 3>{});
        if (++k >= k1) break;
    }
}

// ---------------------------------------------------------------- forces
template <int D, typename T>
__global__ __launch_bounds__(256) void k_force(Dev d, int cur)
{
    const int p = blockIdx.x;
    const DPair &P = d.pairs[p];
    const int a = P.axis, side = -P.sign, dc = P.dc, NV = d.NV;
    const T *f = (const T *)d.f[cur][0];
    int ijk[3];
    ijk[0] = dc % d.n[0];
    ijk[1] = (dc / d.n[0]) % d.n[1];
    ijk[2] = D == 3 ? dc / (d.n[0] * d.n[1]) : 0;
    // F[3] (momentum flux through the face), p_w, tau_w[3], q_n, then the
    // raw moments of the wall distribution (density, momentum, energy)
    double acc[kForceWords] = {};
    for (int k = threadIdx.x; k < NV; k += 256) {
        double xa = d.xi[a][k], st;
        if (side * xa > 0.0) {
            int k1, k2, n1, n2, p1, p2;
            T vm = neighbour(d, f, 0, k, dc, ijk, a, -1, k1, n1, p1);
            T vp = neighbour(d, f, 0, k, dc, ijk, a, +1, k2, n2, p2);
            T v0 = f[(size_t)dc * NV + k];
            st = (double)(v0 + T(side) * T(0.5) * vanleer(v0 - vm, vp - v0)) + fref<T>(d, 0, k);
        } else {
            st = d.face[0][(size_t)p * NV + k];
        }
        double xn = side * xa, dn = 0.0, x2 = 0.0;
        for (int b = 0; b < D; ++b) {
            acc[b] += d.w[k] * d.xi[b][k] * xn * st;
            dn += d.xi[b][k] * P.nw[b];
            x2 += d.xi[b][k] * d.xi[b][k];
        }
        // wall distribution: pressure, tangential stress and normal heat flux
        const double fw = d.fwall[0][(size_t)p * NV + k];
        const double wdf = d.w[k] * dn * fw;
        acc[3] += wdf * dn;
        for (int b = 0; b < D; ++b) acc[4 + b] += wdf * (d.xi[b][k] - dn * P.nw[b]);
        const double e = x2 * fw + (d.NA == 2 ? d.fwall[1][(size_t)p * NV + k] : 0.0);
        acc[7] += 0.5 * d.w[k] * dn * e;
        acc[8] += d.w[k] * fw;
        for (int b = 0; b < D; ++b) acc[9 + b] += d.w[k] * d.xi[b][k] * fw;
        acc[12] += d.w[k] * e;
    }
    for (int b = 0; b < kForceWords; ++b) {
        double s = block_sum(acc[b]);
        if (threadIdx.x == 0) d.pforce[kForceWords * p + b] = b < 3 ? P.dS * s : s;
    }
}

// ---------------------------------------------------------------- state I/O
template <typename T>
__global__ void k_state_from_freestream(Dev d, int buf, int A, const double *u, double amp, long long off, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long g = off + i;
        const int k = (int)(g % d.NV);
        if (sizeof(T) == 4 && d.D == 2 && d.foff)
            ((T *)d.f[buf][A])[g] = (T)(d.fs[A][k] * (u ? amp * u[i] : 0.0));
        else
            ((T *)d.f[buf][A])[g] = (T)(d.fs[A][k] * (1.0 + (u ? amp * u[i] : 0.0)));
    }
}

// freestream times (1 + amp u) with u uniform on (-1, 1) from a counter-based
// generator: the SplitMix64 output function (Steele, Lea and Flood, OOPSLA
// 2014) applied to seed + (index + 1) * golden-ratio increment, index running
// over (array, cell, node) in storage order
__device__ __forceinline__ double hashed_uniform(unsigned long long seed, unsigned long long idx)
{
    unsigned long long z = seed + (idx + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

template <typename T>
__global__ void k_state_hashed(Dev d, int buf, int A, unsigned long long seed, double amp, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(i % d.NV);
        const double u = hashed_uniform(seed, (unsigned long long)A * (unsigned long long)n + (unsigned long long)i);
        if (sizeof(T) == 4 && d.D == 2 && d.foff)
            ((T *)d.f[buf][A])[i] = (T)(d.fs[A][k] * (amp * u));
        else
            ((T *)d.f[buf][A])[i] = (T)(d.fs[A][k] * (1.0 + amp * u));
    }
}

template <typename T>
__global__ void k_state_set(Dev d, int buf, int A, const double *src, long long off, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        ((T *)d.f[buf][A])[off + i] = (T)(src[i] - fref<T>(d, A, (int)((off + i) % d.NV)));
}

template <typename T>
__global__ void k_state_get(Dev d, int buf, int A, double *dst, long long off, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = (double)((const T *)d.f[buf][A])[off + i] + fref<T>(d, A, (int)((off + i) % d.NV));
}

// ---------------------------------------------------------------- measurement
// Streaming copy of n 16-byte words: the practical HBM ceiling the update
// kernels are measured against (every byte read once and written once,
// coalesced 16-byte lanes).  One word per thread, the grid spanning the
// buffer from word base on: on this part this outran grid-stride loops of
// 1 to 8 words per pass and the runtime's copy (6.2 against 4.2-5.4 TB/s).
__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, long long n,
                                                     long long base)
{
    const long long i = base + (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_ctrl_reset(Ctrl *c, int slot)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->tau_bits[slot] = kInfBits;
        c->health = 0u;
    }
}

__global__ void k_moments_out(Dev d, double *out)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.Nc) return;
    const double *cp = d.cellp + (size_t)c * kCellWords;
    double *o = out + (size_t)c * 8;
    if (d.cflag[c] & 1) {
        for (int i = 0; i < 8; ++i) o[i] = NAN;
        return;
    }
    o[0] = cp[CW_RHO];
    for (int a = 0; a < 3; ++a) {
        o[1 + a] = cp[CW_U + a];
        o[5 + a] = cp[CW_Q + a];
    }
    o[4] = cp[CW_T];
}

}  // namespace

#ifndef IBDVM_FP64_UPDATE2D_UNIT

// ---------------------------------------------------------------- allocation-free surface forces
// Scratch of ibdvm_surface_forces_static: the per-pair force records of the
// force kernel (kForceWords doubles per pair, at most kStaticMaxPairs
// pairs), 1.7 MB.  Every device that runs the library holds its own copy
// for the life of the process; calls on one device share it.
static __device__ __align__(256) double scratch[kStaticMaxPairs * kForceWords];

namespace {

// one workgroup: thread 0 sums the force over the pairs in pair order (the
// order of the host sum in ibdvm_surface_forces) and forms C_D, C_L; the
// threads then write the wall points of the first cap pairs
template <int D>
__global__ __launch_bounds__(256) void k_force_out(Dev d, const double *pf, double *out, int cap, double qd,
                                                   double Uinf)
{
    const int np = d.npairs;
    if (threadIdx.x == 0) {
        double F[3] = {0.0, 0.0, 0.0};
        for (int p = 0; p < np; ++p)
            for (int b = 0; b < 3; ++b) F[b] += pf[kForceWords * p + b];
        for (int b = 0; b < 3; ++b) out[b] = F[b];
        out[3] = qd > 0.0 ? F[0] / qd : NAN;
        out[4] = qd > 0.0 ? F[1] / qd : NAN;
    }
    const int m = np < cap ? np : cap;
    for (int p = threadIdx.x; p < m; p += blockDim.x) {
        const DPair &P = d.pairs[p];
        const double *r = pf + kForceWords * p;
        double *w = out + 5 + (size_t)kWallPointWords * p;
        for (int b = 0; b < 3; ++b) {
            w[b] = P.xw[b];
            w[3 + b] = P.nw[b];
            w[8 + b] = r[4 + b];
        }
        w[6] = d.rhow[p];
        w[7] = r[3];
        w[11] = r[7];
        // Section 4: C_p = 2 (p_w - p_0) / (rho_0 U_0^2), freestream p_0 = 1/2
        w[12] = Uinf > 0.0 ? 2.0 * (r[3] - 0.5) / (Uinf * Uinf) : NAN;
        // gas at the wall point: rho, U, then T = 4 (rho E - rho |U|^2 / 2) / (3 rho)
        const double *mw = r + 8;
        double u2 = 0.0;
        for (int b = 0; b < 3; ++b) {
            const double u = b < D ? mw[1 + b] / mw[0] : 0.0;
            w[14 + b] = u;
            u2 += u * u;
        }
        w[13] = 4.0 * (0.5 * mw[4] - 0.5 * mw[0] * u2) / (3.0 * mw[0]);
    }
}

// device address of `scratch` per device, looked up at the first call on a
// device with that device current (the host-side name of the array is not a
// device address)
constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------- launchers
#define DISPATCH(D_, S_, ...)                                      \
    do {                                                           \
        if ((D_) == 2 && (S_) == 0) {                              \
            constexpr int DD = 2;                                  \
            using TT = double;                                     \
            __VA_ARGS__;                                           \
        } else if ((D_) == 2) {                                    \
            constexpr int DD = 2;                                  \
            using TT = float;                                      \
            __VA_ARGS__;                                           \
        } else if ((S_) == 0) {                                    \
            constexpr int DD = 3;                                  \
            using TT = double;                                     \
            __VA_ARGS__;                                           \
        } else {                                                   \
            constexpr int DD = 3;                                  \
            using TT = float;                                      \
            __VA_ARGS__;                                           \
        }                                                          \
    } while (0)

static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }
// grid of a grid-stride loop: a dispatch carries at most 2^32 - 1 work-items
// per dimension, so large element counts loop instead of widening the grid
static inline unsigned stride_blocks(long long n, int bs)
{
    const long long b = (n + bs - 1) / bs;
    return (unsigned)(b < (1ll << 20) ? (b > 0 ? b : 1) : (1ll << 20));
}

hipError_t launch_update2d(const Dev &d, int storage, int cur, int slot, const Tile &t, hipStream_t s)
{
    const int W = 64 * t.V;
    const int ntx = (d.n[0] + t.TX - 1) / t.TX, nys = (d.n[1] + t.LY - 1) / t.LY, ncv = (d.NV + W - 1) / W;
    long long nblk = (long long)ntx * nys * ncv;
    nblk = (nblk + 7) / 8 * 8;
    dim3 grid((unsigned)nblk), block(64 * t.TX);
    if (storage == 0) return launch_update2d_f64(d, t.V, t.TX, cur, slot, t.LY, ntx, nys, ncv, grid, block, s);
#define U2D(VV, XX)                                                                                                   \
    if (t.V == VV && t.TX == XX) {                                                                                 \
        if (d.outer >= kOuterWalls)                                                                                \
            hipLaunchKernelGGL((k_update2d<float, VV, XX, true>), grid, block, 0, s, d, cur, slot, t.LY, ntx, nys, ncv);  \
        else                                                                                                       \
            hipLaunchKernelGGL((k_update2d<float, VV, XX, false>), grid, block, 0, s, d, cur, slot, t.LY, ntx, nys, ncv); \
        return hipGetLastError();                                                                                  \
    }
    U2D(1, 4) U2D(1, 8) U2D(2, 4) U2D(2, 8)
#undef U2D
    return hipErrorInvalidValue;
}

hipError_t launch_update2d_batch(int storage, int V, int TX, bool walls, const BatchArgs &a, hipStream_t s)
{
    long long nblk = a.blk0[a.n];
    if (nblk == 0) return hipSuccess;
    nblk = (nblk + 7) / 8 * 8;
    if (nblk >= (1ll << 31)) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblk), block(64 * TX);
    if (storage == 0) return launch_update2d_batch_f64(V, TX, walls, a, grid, block, s);
#define U2B(VV, XX)                                                                           \
    if (V == VV && TX == XX) {                                                             \
        if (walls)                                                                         \
            hipLaunchKernelGGL((k_update2d_batch<float, VV, XX, true>), grid, block, 0, s, a);  \
        else                                                                               \
            hipLaunchKernelGGL((k_update2d_batch<float, VV, XX, false>), grid, block, 0, s, a); \
        return hipGetLastError();                                                          \
    }
    U2B(1, 4) U2B(1, 8) U2B(2, 4) U2B(2, 8)
#undef U2B
    return hipErrorInvalidValue;
}

hipError_t launch_fill_batch(int D, int storage, const BatchArgs &fin, const BatchArgs &spec, const BatchArgs &ghost,
                             bool implicit, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (fin.blk0[fin.n] > 0) {
        if (implicit)
            DISPATCH(D, storage, hipLaunchKernelGGL((k_fill_fin_batch<DD, TT, true>), dim3((unsigned)fin.blk0[fin.n]), dim3(256), 0, s, fin));
        else
            DISPATCH(D, storage, hipLaunchKernelGGL((k_fill_fin_batch<DD, TT, false>), dim3((unsigned)fin.blk0[fin.n]), dim3(256), 0, s, fin));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (spec.blk0[spec.n] > 0) {
        if (D == 2)
            hipLaunchKernelGGL((k_fill_specular_batch<2>), dim3((unsigned)spec.blk0[spec.n]), dim3(256), 0, s, spec);
        else
            hipLaunchKernelGGL((k_fill_specular_batch<3>), dim3((unsigned)spec.blk0[spec.n]), dim3(256), 0, s, spec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (ghost.blk0[ghost.n] > 0) {
        if (D == 2)
            hipLaunchKernelGGL((k_fill_ghost_batch<2>), dim3((unsigned)ghost.blk0[ghost.n]), dim3(256), 0, s, ghost);
        else
            hipLaunchKernelGGL((k_fill_ghost_batch<3>), dim3((unsigned)ghost.blk0[ghost.n]), dim3(256), 0, s, ghost);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_update3d(const Dev &d, int storage, int cur, int slot, const Tile &t, hipStream_t s)
{
    // t.TX = grid columns per workgroup: 16 (a 4 x 4 tile) or 8 (4 x 2)
    const int TY = t.TX / kT3;
    const int W = 64 * t.V;
    const int ntx = (d.n[0] + kT3 - 1) / kT3, nty = (d.n[1] + TY - 1) / TY, nzs = (d.n[2] + t.LY - 1) / t.LY;
    const int ncv = (d.NV + W - 1) / W;
    long long nblk = (long long)ntx * nty * nzs * ncv;
    nblk = (nblk + 7) / 8 * 8;
    if ((t.TX != 16 && t.TX != 8) || nblk >= (1ll << 31)) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblk), block(64 * t.TX);
#define U3D(TT, VV, YY)                                                                                          \
    if (t.V == VV && TY == YY) {                                                                                 \
        hipLaunchKernelGGL((k_update3d<TT, VV, YY>), grid, block, 0, s, d, cur, slot, t.LY, ntx, nty, nzs, ncv); \
        return hipGetLastError();                                                                                \
    }
    if (storage == 0) {
        U3D(double, 1, 4) U3D(double, 2, 4) U3D(double, 1, 2) U3D(double, 2, 2)
    } else {
        U3D(float, 1, 4) U3D(float, 2, 4) U3D(float, 1, 2) U3D(float, 2, 2)
    }
#undef U3D
    return hipErrorInvalidValue;
}

hipError_t launch_fill_fin(const Dev &d, int storage, int cur, int slot, bool fill, bool fin, hipStream_t s)
{
    const int nfill = fill ? d.npairs * ((d.NV + kFillChunk - 1) / kFillChunk) : 0;
    const bool relax = fin && (d.flags & kFlagImplicit);
    const int nfin = fin ? (int)blocks_for(d.Nc, relax ? kFinCellsRelax : kFinCells) : 0;
    if (nfill + nfin == 0) return hipSuccess;
    if (relax)
        DISPATCH(d.D, storage,
                 hipLaunchKernelGGL((k_fill_fin<DD, TT, true>), dim3(nfill + nfin), dim3(256), 0, s, d, cur, slot, nfill, 1));
    else
        DISPATCH(d.D, storage,
                 hipLaunchKernelGGL((k_fill_fin<DD, TT, false>), dim3(nfill + nfin), dim3(256), 0, s, d, cur, slot, nfill, fin ? 1 : 0));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nfill == 0) return e;
    if (d.alpha < 1.0) {
        if (d.D == 2)
            hipLaunchKernelGGL((k_fill_specular<2>), dim3(nfill), dim3(256), 0, s, d);
        else
            hipLaunchKernelGGL((k_fill_specular<3>), dim3(nfill), dim3(256), 0, s, d);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (d.D == 2)
        hipLaunchKernelGGL((k_fill_ghost<2>), dim3(nfill), dim3(256), 0, s, d);
    else
        hipLaunchKernelGGL((k_fill_ghost<3>), dim3(nfill), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_wall_fill(const Dev &d, int storage, int cur, hipStream_t s)
{
    if (d.outer != kOuterWalls && d.outer != kOuterSpecular) return hipSuccess;
    if (d.D != 2 || !d.wallT[0] || !d.wallT[1]) return hipErrorInvalidValue;
    const dim3 g((unsigned)(2 * (d.n[0] + d.n[1])));
    if (storage == 0)
        hipLaunchKernelGGL((k_wall_fill<double>), g, dim3(256), 0, s, d, cur);
    else
        hipLaunchKernelGGL((k_wall_fill<float>), g, dim3(256), 0, s, d, cur);
    return hipGetLastError();
}

hipError_t launch_moments_direct(const Dev &d, int storage, int cur, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, d.ctrl, slot);
    DISPATCH(d.D, storage, hipLaunchKernelGGL((k_moments_direct<DD, TT>), dim3(blocks_for(d.Nc, 4)), dim3(256), 0, s, d, cur, slot));
    return hipGetLastError();
}

hipError_t launch_force_static(const Dev &d, int storage, int cur, double *out, int cap, double qd, double Uinf,
                               hipStream_t s)
{
    if (d.npairs > kStaticMaxPairs || cap < 0 || !out) return hipErrorInvalidValue;
    void *ptr = nullptr;
    hipError_t e = scratch_address(&ptr);
    if (e != hipSuccess) return e;
    Dev ds = d;
    ds.pforce = (double *)ptr;
    if (d.npairs > 0)
        DISPATCH(d.D, storage, hipLaunchKernelGGL((k_force<DD, TT>), dim3(d.npairs), dim3(256), 0, s, ds, cur));
    if (d.D == 2)
        hipLaunchKernelGGL((k_force_out<2>), dim3(1), dim3(256), 0, s, ds, (const double *)ptr, out, cap, qd, Uinf);
    else
        hipLaunchKernelGGL((k_force_out<3>), dim3(1), dim3(256), 0, s, ds, (const double *)ptr, out, cap, qd, Uinf);
    return hipGetLastError();
}

hipError_t launch_force(const Dev &d, int storage, int cur, hipStream_t s)
{
    if (d.npairs == 0) return hipSuccess;
    DISPATCH(d.D, storage, hipLaunchKernelGGL((k_force<DD, TT>), dim3(d.npairs), dim3(256), 0, s, d, cur));
    return hipGetLastError();
}

hipError_t launch_state_freestream(const Dev &d, int storage, int buf, int A, const double *u, double amp, long long off,
                                   long long n, hipStream_t s)
{
    if (storage == 0)
        hipLaunchKernelGGL(k_state_from_freestream<double>, dim3(stride_blocks(n, 256)), dim3(256), 0, s, d, buf, A, u, amp, off, n);
    else
        hipLaunchKernelGGL(k_state_from_freestream<float>, dim3(stride_blocks(n, 256)), dim3(256), 0, s, d, buf, A, u, amp, off, n);
    return hipGetLastError();
}

hipError_t launch_state_hashed(const Dev &d, int storage, int buf, int A, unsigned long long seed, double amp,
                               hipStream_t s)
{
    const long long n = (long long)d.Nc * d.NV;
    if (storage == 0)
        hipLaunchKernelGGL(k_state_hashed<double>, dim3(stride_blocks(n, 256)), dim3(256), 0, s, d, buf, A, seed, amp, n);
    else
        hipLaunchKernelGGL(k_state_hashed<float>, dim3(stride_blocks(n, 256)), dim3(256), 0, s, d, buf, A, seed, amp, n);
    return hipGetLastError();
}

hipError_t launch_state_set(const Dev &d, int storage, int buf, int A, const double *src, long long off, long long n,
                            hipStream_t s)
{
    if (storage == 0)
        hipLaunchKernelGGL(k_state_set<double>, dim3(stride_blocks(n, 256)), dim3(256), 0, s, d, buf, A, src, off, n);
    else
        hipLaunchKernelGGL(k_state_set<float>, dim3(stride_blocks(n, 256)), dim3(256), 0, s, d, buf, A, src, off, n);
    return hipGetLastError();
}

hipError_t launch_state_get(const Dev &d, int storage, int buf, int A, double *dst, long long off, long long n,
                            hipStream_t s)
{
    if (storage == 0)
        hipLaunchKernelGGL(k_state_get<double>, dim3(stride_blocks(n, 256)), dim3(256), 0, s, d, buf, A, dst, off, n);
    else
        hipLaunchKernelGGL(k_state_get<float>, dim3(stride_blocks(n, 256)), dim3(256), 0, s, d, buf, A, dst, off, n);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, long long words16, hipStream_t s)
{
    // launches of at most 2^30 words (a grid of 2^22 workgroups) each
    constexpr long long kMaxWords = 1ll << 30;
    for (long long base = 0; base < words16; base += kMaxWords) {
        const long long m = std::min(kMaxWords, words16 - base);
        hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, (const uint4 *)src,
                           (uint4 *)dst, base + m, base);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_moments_out(const Dev &d, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments_out, dim3(blocks_for(d.Nc, 256)), dim3(256), 0, s, d, out);
    return hipGetLastError();
}

#else

// The FP64 2D update is compiled in a translation unit of its own
// (IBDVM_FP64_UPDATE2D_UNIT) with the instruction scheduler set to maximise
// instruction-level parallelism, which it gains from and the other kernels
// lose from; that unit defines only these two launchers.
hipError_t launch_update2d_f64(const Dev &d, int V, int TX, int cur, int slot, int LY, int ntx, int nys, int ncv,
                               dim3 grid, dim3 block, hipStream_t s)
{
#define U2D(VV, XX)                                                                                                    \
    if (V == VV && TX == XX) {                                                                                      \
        if (d.outer >= kOuterWalls)                                                                                 \
            hipLaunchKernelGGL((k_update2d<double, VV, XX, true>), grid, block, 0, s, d, cur, slot, LY, ntx, nys, ncv);  \
        else                                                                                                        \
            hipLaunchKernelGGL((k_update2d<double, VV, XX, false>), grid, block, 0, s, d, cur, slot, LY, ntx, nys, ncv); \
        return hipGetLastError();                                                                                   \
    }
    U2D(1, 4) U2D(1, 8) U2D(2, 4) U2D(2, 8)
#undef U2D
    return hipErrorInvalidValue;
}

hipError_t launch_update2d_batch_f64(int V, int TX, bool walls, const BatchArgs &a, dim3 grid, dim3 block, hipStream_t s)
{
#define U2B(VV, XX)                                                                            \
    if (V == VV && TX == XX) {                                                              \
        if (walls)                                                                          \
            hipLaunchKernelGGL((k_update2d_batch<double, VV, XX, true>), grid, block, 0, s, a);  \
        else                                                                                \
            hipLaunchKernelGGL((k_update2d_batch<double, VV, XX, false>), grid, block, 0, s, a); \
        return hipGetLastError();                                                           \
    }
    U2B(1, 4) U2B(1, 8) U2B(2, 4) U2B(2, 8)
#undef U2B
    return hipErrorInvalidValue;
}

#endif

}  // namespace ibdvm
