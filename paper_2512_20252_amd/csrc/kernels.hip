// kernels.hip -- gfx950 kernels of the immersed-boundary Shakhov-DVM step
// (arXiv 2512.20252).  One wavefront owns one cell and 64 consecutive
// velocity nodes (node index innermost in memory, so every load and store of
// the distribution is a contiguous 512-byte (FP64) or 256-byte (FP32) run).
//
//   k_update    Section 2.2 upwind MUSCL fluxes with the van Leer limiter,
//               Shakhov relaxation (Sections 2.1, 4), forward Euler; emits
//               partial moments of the new state per (cell, 64 nodes).
//   k_fill_fin  Section 3.2.1 ghost construction with the upwind weights of
//               3.2.2 and the cut-cell wall density/distribution of 3.2.3,
//               one workgroup per ghost-donor pair; other workgroups of the
//               same launch finish the per-cell moments and tau_min.
//   k_force     momentum flux through the immersed-boundary faces.
//
// Moments of the new state are accumulated about the old bulk velocity U^n
// (peculiar velocity c = xi - U^n, already formed for the equilibrium), so
// the heat flux of the new state follows from shifted raw moments without a
// second pass over the distribution.
#include <hip/hip_runtime.h>

#include <cmath>
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

// van Leer limiter of the hot update: 2 s1 s2 / (s1 + s2) for same-sign
// differences, with the hardware reciprocal refined by Newton steps instead
// of the IEEE division sequence (the result differs by a few ulp)
__device__ __forceinline__ double vl_fast(double s1, double s2)
{
    const double p = s1 * s2, den = s1 + s2;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(fma(-den, r, 1.0), r, r);
    r = fma(fma(-den, r, 1.0), r, r);
    const double sg = 2.0 * s1 * (s2 * r);
    return (p > 0.0 && fabs(den) > 1e-290) ? sg : 0.0;
}

__device__ __forceinline__ float vl_fast(float s1, float s2)
{
    const float p = s1 * s2, den = s1 + s2;
    const float r = __builtin_amdgcn_rcpf(den);
    const float sg = 2.0f * s1 * (s2 * r);
    return (p > 0.0f && fabsf(den) > 1e-35f) ? sg : 0.0f;
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
        if (d.outer == 0) {
            kind = NB_BC;
            nc = -1;
            pr = -1;
            return (T)d.fs[A][k];
        }
        i = (i + d.n[a]) % d.n[a];
    }
    int n = c + (i - ijk[a]) * d.stride[a];
    if (d.cflag[n] & 1) {
        kind = NB_IB;
        nc = -1;
        pr = d.pnb[6 * c + 2 * a + (side > 0 ? 1 : 0)];
        return (T)d.ghost[A][(size_t)pr * d.NV + k];
    }
    kind = NB_FLUID;
    nc = n;
    pr = -1;
    return f[(size_t)n * d.NV + k];
}

// the cell parameters of one fluid cell from its moments; returns tau
__device__ double write_cell(const Dev &d, int c, double rho, const double U[3], double T, const double q[3], int D)
{
    double tau = d.mu0 * pow(T, d.omega) / (0.5 * rho * T);
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
    bool bad = !(rho > 0.0) || !(T > 0.0) || !isfinite(rho) || !isfinite(T) || !isfinite(tau);
    if (bad) atomicOr(&d.ctrl->health, 1u);
    return bad ? INFINITY : tau;
}

__device__ __forceinline__ void tau_min_commit(const Dev &d, int slot, double tau)
{
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) tau = fmin(tau, __shfl_xor(tau, m, 64));
    if (lane == 0) red[wv] = tau;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
        if (t < INFINITY) atomicMin(&d.ctrl->tau_bits[slot], (unsigned long long)__double_as_longlong(t));
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
__device__ double vel_interp(const Dev &d, const double *g, const double v[3], int D)
{
    int i0[3] = {0, 0, 0};
    double t[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
        const double *x = d.xa + a * kMaxVn;
        int N = d.vn[a];
        if (v[a] < x[0] || v[a] > x[N - 1]) return 0.0;
        int i = (int)floor((v[a] - x[0]) / (x[1] - x[0]));
        i = i < 0 ? 0 : (i > N - 2 ? N - 2 : i);
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
template <int D, typename T>
__device__ void fill_pair(const Dev &d, int cur, int p)
{
    const DPair &P = d.pairs[p];
    const int a = P.axis, dc = P.dc, ac = P.ac, ns = P.ns;
    const double ygc = P.ygc, ydc = P.ydc, yac = P.yac, yw = P.yw, ysp = P.ysp, yface = P.yface;
    const size_t po = (size_t)p * d.NV;
    const int NV = d.NV;
    const bool uniform = (d.flags & 2u) != 0;  // NO_UPWIND ablation
    double num = 0.0;
    for (int A = 0; A < d.NA; ++A) {
        const T *f = (const T *)d.f[cur][A];
        for (int k = threadIdx.x; k < NV; k += 256) {
            double xk[3] = {0, 0, 0}, x2 = 0.0;
            for (int b = 0; b < D; ++b) {
                xk[b] = d.xi[b][k];
                x2 += xk[b] * xk[b];
            }
            // 1. shifted point from the donor and the auxiliary-cell slope
            double fdc = (double)f[(size_t)dc * NV + k];
            double sdc = ac >= 0 ? ((double)f[(size_t)ac * NV + k] - fdc) / (yac - ydc) : 0.0;
            double fspv = fdc + sdc * (ysp - ydc);
            // 2. upwind-weighted interpolation from the surface cells
            double thr = 1e-12 * sqrt(x2), sum = 0.0;
            for (int j = 0; j < ns; ++j) {
                double dd = 0.0;
                for (int b = 0; b < D; ++b) dd += xk[b] * P.rh[j][b];
                if (fabs(dd) <= thr) dd = 0.0;
                double m = dd < 0.0 ? -dd : 0.0;
                sum += m * m;
            }
            double fgc = 0.0;
            for (int j = 0; j < ns; ++j) {
                double wj;
                if (uniform || sum == 0.0) {
                    wj = 1.0 / ns;
                } else {
                    double dd = 0.0;
                    for (int b = 0; b < D; ++b) dd += xk[b] * P.rh[j][b];
                    if (fabs(dd) <= thr) dd = 0.0;
                    double m = dd < 0.0 ? -dd : 0.0;
                    wj = m * m / sum;
                }
                const int sj = P.sc[j];
                double fj = (double)f[(size_t)sj * NV + k], sr = 0.0;
                for (int b = 0; b < D; ++b) {
                    int L = P.snb[j][b][0], R = P.snb[j][b][1];
                    double sg = 0.0;
                    if (L >= 0 && R >= 0)
                        sg = vanleer(fj - (double)f[(size_t)L * NV + k], (double)f[(size_t)R * NV + k] - fj) * d.inv_dx[b];
                    else if (R >= 0)
                        sg = ((double)f[(size_t)R * NV + k] - fj) * d.inv_dx[b];
                    else if (L >= 0)
                        sg = (fj - (double)f[(size_t)L * NV + k]) * d.inv_dx[b];
                    sr += sg * P.r[j][b];
                }
                fgc += wj * (fj - sr);
            }
            // 3. incident distribution at the intersect point
            double fiw = fspv + (fgc - fspv) / (ygc - ysp) * (yw - ysp);
            d.fiw[A][po + k] = fiw;
            d.fsp[A][po + k] = fspv;
            if (A == 0) {
                double dn = 0.0;
                for (int b = 0; b < D; ++b) dn += xk[b] * P.nw[b];
                int cl = d.cls[po + k];
                double wt = cl == 0 ? d.w[k] : (cl >= 2 ? d.wg[po + k] : 0.0);
                num += wt * dn * fiw;
            }
        }
    }
    __threadfence_block();
    __syncthreads();
    const double al = d.alpha;
    if (al < 1.0) {
        for (int k = threadIdx.x; k < NV; k += 256) {
            int cl = d.cls[po + k];
            if (cl == 0) continue;
            double xk[3] = {0, 0, 0}, dn = 0.0;
            for (int b = 0; b < D; ++b) {
                xk[b] = d.xi[b][k];
                dn += xk[b] * P.nw[b];
            }
            double v[3] = {0, 0, 0};
            for (int b = 0; b < D; ++b) v[b] = xk[b] - 2.0 * dn * P.nw[b];
            double fsv = vel_interp(d, d.fiw[0] + po, v, D);
            double ws = cl == 1 ? d.w[k] : d.w[k] - d.wg[po + k];
            num += (1.0 - al) * ws * dn * fsv;
        }
    }
    num = block_sum(num);
    const double rw = al > 0.0 ? -num / (al * P.den) : 0.0;
    if (threadIdx.x == 0) d.rhow[p] = rw;
    for (int A = 0; A < d.NA; ++A) {
        for (int k = threadIdx.x; k < NV; k += 256) {
            int cl = d.cls[po + k];
            double fi = d.fiw[A][po + k];
            double fsv = 0.0;
            if (al < 1.0 && cl != 0) {
                double xk[3] = {0, 0, 0}, dn = 0.0;
                for (int b = 0; b < D; ++b) {
                    xk[b] = d.xi[b][k];
                    dn += xk[b] * P.nw[b];
                }
                double v[3] = {0, 0, 0};
                for (int b = 0; b < D; ++b) v[b] = xk[b] - 2.0 * dn * P.nw[b];
                fsv = vel_interp(d, d.fiw[A] + po, v, D);
            }
            double Hw = d.hw[k] * (A == 1 ? 0.5 * d.Tw : 1.0);
            double fr = al * rw * Hw + (1.0 - al) * fsv;
            double fw = cl == 0 ? fi : (cl == 1 ? fr : (d.wg[po + k] * fi + (d.w[k] - d.wg[po + k]) * fr) / d.w[k]);
            double fspv = d.fsp[A][po + k];
            double sig = (fw - fspv) / (yw - ysp);
            double gv = fspv + sig * (ygc - ysp);
            d.ghost[A][po + k] = gv;
            d.face[A][po + k] = gv + sig * (yface - ygc);
        }
    }
}

// ---------------------------------------------------------------- moments
template <int D>
__device__ void fin_cells(const Dev &d, int slot, int blk)
{
    constexpr int PW = D == 2 ? kPartialWords2 : kPartialWords3;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double tmin = INFINITY;
    for (int i = 0; i < 8; ++i) {
        const int c = blk * 32 + wv * 8 + i;
        if (c >= d.Nc) break;
        if (d.cflag[c] & 1) continue;
        double acc = 0.0;
        if (lane < PW)
            for (int ch = 0; ch < d.nchunk; ++ch) acc += d.part[((size_t)c * d.nchunk + ch) * kPartialStride + lane];
        double S[PW];
#pragma unroll
        for (int j = 0; j < PW; ++j) S[j] = __shfl(acc, j, 64);
        const double *cp = d.cellp + (size_t)c * kCellWords;
        double Uref[3] = {cp[CW_U], cp[CW_U + 1], cp[CW_U + 2]};
        double m0 = S[0], m1[3] = {0, 0, 0}, m3[3] = {0, 0, 0}, M[3][3] = {};
        for (int a = 0; a < D; ++a) {
            m1[a] = S[1 + a];
            m3[a] = S[2 + D + a];
        }
        double m2 = S[1 + D];
        int o = 2 + 2 * D;
        for (int a = 0; a < D; ++a)
            for (int b = a; b < D; ++b) {
                M[a][b] = M[b][a] = S[o];
                ++o;
            }
        double del[3] = {0, 0, 0}, U[3] = {0, 0, 0}, mm = 0.0, dd = 0.0;
        for (int a = 0; a < D; ++a) {
            del[a] = m1[a] / m0;
            U[a] = Uref[a] + del[a];
            mm += m1[a] * m1[a];
            dd += del[a] * del[a];
        }
        double T = (2.0 / 3.0) * (m2 - mm / m0) / m0;
        double q[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            double Md = 0.0;
            for (int b = 0; b < D; ++b) Md += M[a][b] * del[b];
            q[a] = 0.5 * (m3[a] - 2.0 * Md - del[a] * m2 + 2.0 * dd * m1[a]);
        }
        double tau = INFINITY;
        if (lane == 0) tau = write_cell(d, c, m0, U, T, q, D);
        tmin = fmin(tmin, tau);
    }
    tau_min_commit(d, slot, tmin);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_fill_fin(Dev d, int cur, int slot, int nfill, int dofin)
{
    if ((int)blockIdx.x < nfill) {
        fill_pair<D, T>(d, cur, blockIdx.x);
        return;
    }
    if (dofin) fin_cells<D>(d, slot, blockIdx.x - nfill);
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
            double h = (double)f0[k], x2 = 0.0;
            for (int a = 0; a < D; ++a) {
                double x = d.xi[a][k];
                x2 += x * x;
                m[a] += d.w[k] * x * h;
            }
            rho += d.w[k] * h;
            E2 += d.w[k] * (x2 * h + (D == 2 ? (double)f1[k] : 0.0));
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
            double E = c2 * (double)f0[k] + (D == 2 ? (double)f1[k] : 0.0);
            for (int a = 0; a < D; ++a) q[a] += d.w[k] * cc[a] * E;
        }
        for (int a = 0; a < D; ++a) q[a] = 0.5 * wave_sum(q[a]);
        if (lane == 0) tau = write_cell(d, c, rho, U, Tc, q, D);
    }
    tau_min_commit(d, slot, tau);
}

// ---------------------------------------------------------------- update
template <int D, typename T>
__global__ __launch_bounds__(256) void k_update(Dev d, int cur, int slot)
{
    constexpr int PW = D == 2 ? kPartialWords2 : kPartialWords3;
    const int lane = threadIdx.x & 63;
    const double tmin = __longlong_as_double((long long)d.ctrl->tau_bits[slot]);
    const double dt = d.cfl / (d.adv + 1.0 / tmin);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.ctrl->tau_bits[slot ^ 1] = kInfBits;
        d.ctrl->dt = dt;
        d.ctrl->time += dt;
        d.ctrl->step += 1;
    }
    const long long wave = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= (long long)d.Nc * d.nchunk) return;
    const int c = (int)(wave / d.nchunk), chunk = (int)(wave - (long long)c * d.nchunk);
    const int fl = d.cflag[c];
    const int NV = d.NV;
    const int k = chunk * kChunk + lane;
    const bool act = k < NV;
    const int kk = act ? k : NV - 1;
    if (fl & 1) {
        // solid cells are not advanced; carry their value into the new buffer
        if (act)
            for (int A = 0; A < d.NA; ++A)
                ((T *)d.f[cur ^ 1][A])[(size_t)c * NV + k] = ((const T *)d.f[cur][A])[(size_t)c * NV + k];
        return;
    }
    int ijk[3];
    ijk[0] = c % d.n[0];
    ijk[1] = (c / d.n[0]) % d.n[1];
    ijk[2] = D == 3 ? c / (d.n[0] * d.n[1]) : 0;

    const double *cp = d.cellp + (size_t)c * kCellWords;
    double cc[3] = {0, 0, 0}, c2 = 0.0, cs = 0.0, xi[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
        xi[a] = d.xi[a][kk];
        cc[a] = xi[a] - cp[CW_U + a];
        c2 += cc[a] * cc[a];
        cs += cc[a] * cp[CW_S + a];
    }
    const double invT = cp[CW_INVT];
    const double H = cp[CW_A] * exp(-c2 * invT);
    double gS[2];
    if (D == 2) {
        gS[0] = H * (1.0 + cs * (2.0 * c2 * invT - 4.0));
        gS[1] = cp[CW_TH] * H * (1.0 + cs * (2.0 * c2 * invT - 2.0));
    } else {
        gS[0] = H * (1.0 + cs * (2.0 * c2 * invT - 5.0));
        gS[1] = 0.0;
    }
    const double rate = dt * cp[CW_INVTAU];
    double fnew[2] = {0.0, 0.0};
    for (int A = 0; A < d.NA; ++A) {
        const T *f = (const T *)d.f[cur][A];
        const T v0 = f[(size_t)c * NV + kk];
        T div = T(0);
        for (int a = 0; a < D; ++a) {
            T vm2, vm1, vp1, vp2;
            int km1 = NB_FLUID, kp1 = NB_FLUID, pm1 = -1, pp1 = -1;
            if (!(fl & 2)) {
                const size_t s = (size_t)d.stride[a] * NV, o = (size_t)c * NV + kk;
                vm2 = f[o - 2 * s];
                vm1 = f[o - s];
                vp1 = f[o + s];
                vp2 = f[o + 2 * s];
            } else {
                int nm, np, dummy, kind2;
                vm1 = neighbour(d, f, A, kk, c, ijk, a, -1, km1, nm, pm1);
                vp1 = neighbour(d, f, A, kk, c, ijk, a, +1, kp1, np, pp1);
                vm2 = vm1;
                vp2 = vp1;
                if (km1 == NB_FLUID) {
                    int j2[3] = {ijk[0], ijk[1], ijk[2]};
                    j2[a] = (ijk[a] - 1 + d.n[a]) % d.n[a];
                    vm2 = neighbour(d, f, A, kk, nm, j2, a, -1, kind2, dummy, dummy);
                }
                if (kp1 == NB_FLUID) {
                    int j2[3] = {ijk[0], ijk[1], ijk[2]};
                    j2[a] = (ijk[a] + 1) % d.n[a];
                    vp2 = neighbour(d, f, A, kk, np, j2, a, +1, kind2, dummy, dummy);
                }
            }
            const T s0 = vanleer(v0 - vm1, vp1 - v0);
            const T xa = (T)xi[a];
            T fr, fl_;
            if (xa > T(0)) {
                fr = v0 + T(0.5) * s0;
                if (km1 == NB_IB)
                    fl_ = (T)d.face[A][(size_t)pm1 * NV + kk];
                else if (km1 == NB_BC)
                    fl_ = vm1;
                else
                    fl_ = vm1 + T(0.5) * vanleer(vm1 - vm2, v0 - vm1);
            } else {
                fl_ = v0 - T(0.5) * s0;
                if (kp1 == NB_IB)
                    fr = (T)d.face[A][(size_t)pp1 * NV + kk];
                else if (kp1 == NB_BC)
                    fr = vp1;
                else
                    fr = vp1 - T(0.5) * vanleer(vp1 - v0, vp2 - vp1);
            }
            div += xa * (fr - fl_) * (T)d.inv_dx[a];
        }
        const double fo = (double)v0;
        const double fn = fo - dt * (double)div + rate * (gS[A] - fo);
        const T st = (T)fn;
        if (act) ((T *)d.f[cur ^ 1][A])[(size_t)c * NV + k] = st;
        fnew[A] = act ? (double)st : 0.0;
    }
    // partial moments of the new state about U^n
    const double wk = act ? d.w[k] : 0.0;
    const double h = fnew[0];
    const double E = c2 * h + (D == 2 ? fnew[1] : 0.0);
    double S[PW];
    S[0] = wk * h;
    for (int a = 0; a < D; ++a) {
        S[1 + a] = wk * cc[a] * h;
        S[2 + D + a] = wk * cc[a] * E;
    }
    S[1 + D] = wk * E;
    int o = 2 + 2 * D;
    for (int a = 0; a < D; ++a)
        for (int b = a; b < D; ++b) S[o++] = wk * cc[a] * cc[b] * h;
    double mine = 0.0;
#pragma unroll
    for (int j = 0; j < PW; ++j) {
        double v = wave_sum(S[j]);
        if (lane == j) mine = v;
    }
    if (lane < PW) d.part[((size_t)c * d.nchunk + chunk) * kPartialStride + lane] = mine;
}

// ---------------------------------------------------------------- 2D update, marching in y
// Workgroup = TX wavefronts; wavefront w owns grid column i0 + w and its lanes
// own velocity nodes k0 + lane + 64 v (v < V).  The workgroup marches up a
// segment of rows.  Rows j-2..j+2 of the own column live in registers; row j
// of the TX columns plus two halo columns per side is exchanged through LDS
// (double-buffered by row parity), the x slopes of the TX + 2 cells the faces
// need are computed once per row and shared through LDS, and the y slope of
// row j+1 and the flux state of face j+1/2 are carried to the next row.  Outer
// freestream ghosts are the freestream values (zero slope follows from the
// limiter); periodic ghosts wrap.  Solid face neighbours are replaced by the
// ghost value of the pair seen from the fluid cell, and faces toward a solid
// cell take the pair's ghost-side face value.

// sums S[0..8] over the 64 lanes; lane 8m holds the total of S[m] for m < 8,
// every lane holds the total of S[8].  Three exchange steps halve the number
// of values each lane carries, three more finish the lane sum.
__device__ __forceinline__ void reduce9(const double S[9], double &r8, double &s8)
{
    const int lane = threadIdx.x & 63;
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
    double a[4], b[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double keep = b5 ? S[4 + i] : S[i];
        double send = b5 ? S[i] : S[4 + i];
        a[i] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        double keep = b4 ? a[2 + i] : a[i];
        double send = b4 ? a[i] : a[2 + i];
        b[i] = keep + __shfl_xor(send, 16, 64);
    }
    double keep = b3 ? b[1] : b[0];
    double send = b3 ? b[0] : b[1];
    double c = keep + __shfl_xor(send, 8, 64);
    c += __shfl_xor(c, 4, 64);
    c += __shfl_xor(c, 2, 64);
    c += __shfl_xor(c, 1, 64);
    r8 = c;
    s8 = wave_sum(S[8]);
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
__device__ __forceinline__ double unid(double x)
{
    long long b = __double_as_longlong(x);
    int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// start of the node row of cell (ic, jr); outer freestream ghosts read the
// freestream row, periodic ghosts wrap
template <typename T>
__device__ __forceinline__ const T *row_of(const Dev &d, const T *f, const T *fsT, int ic, int jr)
{
    const int nx = d.n[0], ny = d.n[1];
    if ((unsigned)ic >= (unsigned)nx || (unsigned)jr >= (unsigned)ny) {
        if (d.outer == 0) return fsT;
        ic = (ic + nx) % nx;
        jr = (jr + ny) % ny;
    }
    return f + (size_t)(ic + nx * jr) * d.NV;
}

// read-only tables indexed by wavefront-uniform values go through the
// scalar cache (constant address space): the loads land in scalar registers
// and are counted apart from the vector loads still in flight
typedef const __attribute__((address_space(4))) int *cint_p;
typedef const __attribute__((address_space(4))) double *cdbl_p;

__device__ __forceinline__ int flags_at(const Dev &d, int ic, int jr)
{
    if ((unsigned)ic >= (unsigned)d.n[0] || (unsigned)jr >= (unsigned)d.n[1]) return 0;
    return ((cint_p)d.cflag)[ic + d.n[0] * jr];
}

// ghost value / ghost-side face value of the pair seen from fluid cell c in
// direction dir (2 axis + side)
template <typename T>
__device__ __forceinline__ T ghost_of(const Dev &d, int A, int c, int dir, int kk)
{
    const int p = ((cint_p)d.pnb)[6 * c + dir];
    return (T)d.ghost[A][(size_t)p * d.NV + kk];
}

template <typename T>
__device__ __forceinline__ T facev_of(const Dev &d, int A, int c, int dir, int kk)
{
    const int p = ((cint_p)d.pnb)[6 * c + dir];
    return (T)d.face[A][(size_t)p * d.NV + kk];
}

template <typename T, int V, int TX>
__global__ __launch_bounds__(TX * 64) void k_update2d(Dev d, int cur, int slot, int LY, int ntx, int nys, int ncv)
{
    constexpr int W = 64 * V;
    // row j of the tile's columns and two halo columns per side (by row
    // parity), and the outgoing x-face state of the TX + 2 cells the faces
    // need: f + sigma/2 where xi_x > 0, f - sigma/2 otherwise
    __shared__ T fb[2][2][TX + 4][W];
    __shared__ T ob[2][TX + 2][W];

    const double tmin = __longlong_as_double((long long)d.ctrl->tau_bits[slot]);
    const double dt = d.cfl / (d.adv + 1.0 / tmin);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.ctrl->tau_bits[slot ^ 1] = kInfBits;
        d.ctrl->dt = dt;
        d.ctrl->time += dt;
        d.ctrl->step += 1;
    }
    // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of tiles so that x-neighbouring tiles share its L2
    const int nb = gridDim.x;
    const int L = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    if (L >= ntx * nys * ncv) return;
    const int tx = L % ntx, ys = (L / ntx) % nys, ch = L / (ntx * nys);
    const int nx = d.n[0], ny = d.n[1], NV = d.NV;
    const int i0 = tx * TX, j0 = ys * LY, j1 = min(j0 + LY, ny);
    const int lane = threadIdx.x & 63;
    const int w = uni(threadIdx.x >> 6);
    const int i = i0 + w;
    const bool col_in = i < nx;

    int kk[V];
    bool act[V], pos[V];
    double xx[V], xy[V], wk[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        int k = ch * W + v * 64 + lane;
        act[v] = k < NV;
        kk[v] = act[v] ? k : NV - 1;
        xx[v] = d.xi[0][kk[v]];
        xy[v] = d.xi[1][kk[v]];
        wk[v] = act[v] ? d.w[kk[v]] : 0.0;
        pos[v] = xx[v] > 0.0;
    }
    const T *fA[2] = {(const T *)d.f[cur][0], (const T *)d.f[cur][1]};
    T *gA[2] = {(T *)d.f[cur ^ 1][0], (T *)d.f[cur ^ 1][1]};
    const T *fsT[2] = {(const T *)d.fsT[0], (const T *)d.fsT[1]};
    const T hdx = T(0.5);
    const double idx = d.inv_dx[0], idy = d.inv_dx[1];

    // halo columns loaded by wavefronts 0..3, halo face states made by 0..1
    const int hcol = w < 2 ? i0 - 2 + w : i0 + TX + (w - 2);
    const int hpos = w < 2 ? w : TX + 2 + (w - 2);
    const int scol = w == 0 ? i0 - 1 : i0 + TX;
    const int spos = w == 0 ? 0 : TX + 1;

    auto flag_row = [&](int m) -> int { return col_in ? flags_at(d, i, m) : 0; };
    auto flag_halo = [&](int m) -> int { return flags_at(d, scol, m); };

    // y slope of cell (i, m) from rows m-1, m, m+1 with ghost substitution
    auto slope_y = [&](int A, int v, T fm, T f0, T fp, int m, int fl) -> T {
        if (fl & CF_SOLID) return T(0);
        if (fl & (CF_YM | CF_YP)) {
            const int c = i + nx * m;
            if (fl & CF_YM) fm = ghost_of<T>(d, A, c, 2, kk[v]);
            if (fl & CF_YP) fp = ghost_of<T>(d, A, c, 3, kk[v]);
        }
        return vl_fast(f0 - fm, fp - f0);
    };
    // upwind state of the face between rows m (below) and m+1 (above)
    auto face_y = [&](int A, int v, T fl_, T sl_, int flL, T fr_, T sr_, int flR, int m) -> T {
        if (xy[v] > 0.0) {
            if (!(flL & CF_SOLID)) return fl_ + hdx * sl_;
            if (flR & CF_SOLID) return T(0);
            return facev_of<T>(d, A, i + nx * (m + 1), 2, kk[v]);
        }
        if (!(flR & CF_SOLID)) return fr_ - hdx * sr_;
        if (flL & CF_SOLID) return T(0);
        return facev_of<T>(d, A, i + nx * m, 3, kk[v]);
    };

    // rows j-1..j+2 of the own column; the row after next, the next halo row
    // and the next cell's equilibrium parameters are fetched one row ahead
    T q[2][4][V], nxt[2][V], hnx[2][V];
    double cpn[8];
    auto fetch_cell = [&](int m) {
        const cdbl_p cp = (cdbl_p)d.cellp + (size_t)(col_in ? i + nx * m : 0) * kCellWords;
        cpn[0] = cp[CW_U];
        cpn[1] = cp[CW_U + 1];
        cpn[2] = cp[CW_A];
        cpn[3] = cp[CW_INVT];
        cpn[4] = cp[CW_S];
        cpn[5] = cp[CW_S + 1];
        cpn[6] = cp[CW_TH];
        cpn[7] = cp[CW_INVTAU];
    };
    T s0[2][V], Fdn[2][V];
    {
        T qm2[2][V];
#pragma unroll
        for (int A = 0; A < 2; ++A) {
            const T *r0 = row_of(d, fA[A], fsT[A], i, j0 - 2);
            const T *r1 = row_of(d, fA[A], fsT[A], i, j0 - 1);
            const T *r2 = row_of(d, fA[A], fsT[A], i, j0);
            const T *r3 = row_of(d, fA[A], fsT[A], i, j0 + 1);
            const T *rp = row_of(d, fA[A], fsT[A], i, j0 + 2);
            const T *hp = row_of(d, fA[A], fsT[A], hcol, j0);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                qm2[A][v] = r0[kk[v]];
                q[A][0][v] = r1[kk[v]];
                q[A][1][v] = r2[kk[v]];
                q[A][2][v] = r3[kk[v]];
                nxt[A][v] = rp[kk[v]];
                hnx[A][v] = w < 4 ? hp[kk[v]] : T(0);
            }
        }
        fetch_cell(j0);
        const int flm1 = flag_row(j0 - 1), fl0i = flag_row(j0);
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                T sm = slope_y(A, v, qm2[A][v], q[A][0][v], q[A][1][v], j0 - 1, flm1);
                s0[A][v] = slope_y(A, v, q[A][0][v], q[A][1][v], q[A][2][v], j0, fl0i);
                Fdn[A][v] = face_y(A, v, q[A][0][v], sm, flm1, q[A][1][v], s0[A][v], fl0i, j0 - 1);
            }
    }
    int fl0 = flag_row(j0);

    for (int j = j0; j < j1; ++j) {
        const int buf = (j - j0) & 1;
        // q[A][1] is row j, q[A][2] row j+1, q[A][3] row j+2
        T hcur[2][V];
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                q[A][3][v] = nxt[A][v];
                hcur[A][v] = hnx[A][v];
            }
        // equilibrium parameters of cell (i, j), wavefront-uniform
        const double U0 = cpn[0], U1 = cpn[1], Ac = cpn[2], invT = cpn[3];
        const double S0 = cpn[4], S1 = cpn[5], Th = cpn[6], itau = cpn[7];
        if (j + 1 < j1) {
#pragma unroll
            for (int A = 0; A < 2; ++A) {
                const T *rp = row_of(d, fA[A], fsT[A], i, j + 3);
#pragma unroll
                for (int v = 0; v < V; ++v) nxt[A][v] = rp[kk[v]];
                if (w < 4) {
                    const T *hp = row_of(d, fA[A], fsT[A], hcol, j + 1);
#pragma unroll
                    for (int v = 0; v < V; ++v) hnx[A][v] = hp[kk[v]];
                }
            }
            fetch_cell(j + 1);
        }
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                fb[buf][A][w + 2][v * 64 + lane] = q[A][1][v];
                if (w < 4) fb[buf][A][hpos][v * 64 + lane] = hcur[A][v];
            }
        lds_barrier();
        // outgoing x-face states of the own cell and of the halo cell
        T own_out[2][V];
        {
            const int c = i + nx * j;
            auto run = [&](auto near_tag) {
                constexpr bool NEAR = decltype(near_tag)::value;
#pragma unroll
                for (int A = 0; A < 2; ++A)
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        T fm = fb[buf][A][w + 1][v * 64 + lane];
                        T fp = fb[buf][A][w + 3][v * 64 + lane];
                        const T f0 = q[A][1][v];
                        if (NEAR && (fl0 & CF_XM)) fm = ghost_of<T>(d, A, c, 0, kk[v]);
                        if (NEAR && (fl0 & CF_XP)) fp = ghost_of<T>(d, A, c, 1, kk[v]);
                        T s = vl_fast(f0 - fm, fp - f0);
                        if (NEAR && (fl0 & CF_SOLID)) s = T(0);
                        const T o = pos[v] ? f0 + hdx * s : f0 - hdx * s;
                        own_out[A][v] = o;
                        ob[A][w + 1][v * 64 + lane] = o;
                    }
            };
            if (fl0 & (CF_SOLID | CF_XM | CF_XP))
                run(std::true_type{});
            else
                run(std::false_type{});
        }
        if (w < 2) {
            const int fl = flag_halo(j);
            const int c = scol + nx * j;
            auto run = [&](auto near_tag) {
                constexpr bool NEAR = decltype(near_tag)::value;
#pragma unroll
                for (int A = 0; A < 2; ++A)
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        T fm = fb[buf][A][spos][v * 64 + lane];
                        const T f0 = fb[buf][A][spos + 1][v * 64 + lane];
                        T fp = fb[buf][A][spos + 2][v * 64 + lane];
                        if (NEAR && (fl & CF_XM)) fm = ghost_of<T>(d, A, c, 0, kk[v]);
                        if (NEAR && (fl & CF_XP)) fp = ghost_of<T>(d, A, c, 1, kk[v]);
                        T s = vl_fast(f0 - fm, fp - f0);
                        if (NEAR && (fl & CF_SOLID)) s = T(0);
                        ob[A][spos][v * 64 + lane] = pos[v] ? f0 + hdx * s : f0 - hdx * s;
                    }
            };
            if (fl & (CF_SOLID | CF_XM | CF_XP))
                run(std::true_type{});
            else
                run(std::false_type{});
        }
        lds_barrier();

        const int flp1 = flag_row(j + 1);
        const int c = i + nx * j;
        const bool upd = col_in && !(fl0 & CF_SOLID);
        double mom[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        const double rate = dt * itau;
        T *g0 = gA[0] + (size_t)c * NV, *g1 = gA[1] + (size_t)c * NV;
        auto run = [&](auto near_tag) {
            constexpr bool NEAR = decltype(near_tag)::value;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                T s1[2];
                T Fup[2];
#pragma unroll
                for (int A = 0; A < 2; ++A) {
                    if (NEAR) {
                        s1[A] = slope_y(A, v, q[A][1][v], q[A][2][v], q[A][3][v], j + 1, flp1);
                        Fup[A] = face_y(A, v, q[A][1][v], s0[A][v], fl0, q[A][2][v], s1[A], flp1, j);
                    } else {
                        const T fm = q[A][1][v], f0 = q[A][2][v], fp = q[A][3][v];
                        s1[A] = vl_fast(f0 - fm, fp - f0);
                        Fup[A] = xy[v] > 0.0 ? fm + hdx * s0[A][v] : f0 - hdx * s1[A];
                    }
                }
                if (upd) {
                    const double cx = xx[v] - U0, cy = xy[v] - U1;
                    const double c2 = cx * cx + cy * cy, cs = cx * S0 + cy * S1;
                    const double H = Ac * exp(-c2 * invT);
                    const double gS[2] = {H * (1.0 + cs * (2.0 * c2 * invT - 4.0)),
                                          Th * H * (1.0 + cs * (2.0 * c2 * invT - 2.0))};
                    double fnew[2];
#pragma unroll
                    for (int A = 0; A < 2; ++A) {
                        const T f0 = q[A][1][v];
                        // the neighbour's outgoing state is the face state on the upwind side
                        const T nb = ob[A][pos[v] ? w : w + 2][v * 64 + lane];
                        T Fr, Fl;
                        if (pos[v]) {
                            Fr = own_out[A][v];
                            Fl = (NEAR && (fl0 & CF_XM)) ? facev_of<T>(d, A, c, 0, kk[v]) : nb;
                        } else {
                            Fl = own_out[A][v];
                            Fr = (NEAR && (fl0 & CF_XP)) ? facev_of<T>(d, A, c, 1, kk[v]) : nb;
                        }
                        const T div = (T)xx[v] * (Fr - Fl) * (T)idx + (T)xy[v] * (Fup[A] - Fdn[A][v]) * (T)idy;
                        const double fo = (double)f0;
                        const T st = (T)(fo - dt * (double)div + rate * (gS[A] - fo));
                        if (act[v]) (A == 0 ? g0 : g1)[kk[v]] = st;
                        fnew[A] = act[v] ? (double)st : 0.0;
                    }
                    const double wh = wk[v] * fnew[0], wE = wk[v] * (c2 * fnew[0] + fnew[1]);
                    const double tx_ = cx * wh, ty_ = cy * wh;
                    mom[0] += wh;
                    mom[1] += tx_;
                    mom[2] += ty_;
                    mom[3] += wE;
                    mom[4] += cx * wE;
                    mom[5] += cy * wE;
                    mom[6] += cx * tx_;
                    mom[7] += cy * tx_;
                    mom[8] += cy * ty_;
                } else if (col_in && act[v]) {
                    // solid cells are not advanced; carry their value
                    g0[kk[v]] = q[0][1][v];
                    g1[kk[v]] = q[1][1][v];
                }
#pragma unroll
                for (int A = 0; A < 2; ++A) {
                    Fdn[A][v] = Fup[A];
                    s0[A][v] = s1[A];
                }
            }
        };
        if ((fl0 | flp1) & (CF_SOLID | CF_XM | CF_XP | CF_YM | CF_YP))
            run(std::true_type{});
        else
            run(std::false_type{});
        if (upd) {
            // partial record: m0, m1x, m1y, m2, m3x, m3y, Mxx, Mxy, Myy
            double r8, s8;
            reduce9(mom, r8, s8);
            double *pp = d.part + ((size_t)c * ncv + ch) * kPartialStride;
            if ((lane & 7) == 0) pp[lane >> 3] = r8;
            if (lane == 1) pp[8] = s8;
        }
        fl0 = flp1;
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                q[A][0][v] = q[A][1][v];
                q[A][1][v] = q[A][2][v];
                q[A][2][v] = q[A][3][v];
            }
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
    double acc[4] = {0, 0, 0, 0};
    const double ygc = P.ygc, yw = P.yw, ysp = P.ysp;
    for (int k = threadIdx.x; k < NV; k += 256) {
        double xa = d.xi[a][k], st;
        if (side * xa > 0.0) {
            int k1, k2, n1, n2, p1, p2;
            T vm = neighbour(d, f, 0, k, dc, ijk, a, -1, k1, n1, p1);
            T vp = neighbour(d, f, 0, k, dc, ijk, a, +1, k2, n2, p2);
            T v0 = f[(size_t)dc * NV + k];
            st = (double)(v0 + T(side) * T(0.5) * vanleer(v0 - vm, vp - v0));
        } else {
            st = d.face[0][(size_t)p * NV + k];
        }
        double xn = side * xa, dn = 0.0;
        for (int b = 0; b < D; ++b) {
            acc[b] += d.w[k] * d.xi[b][k] * xn * st;
            dn += d.xi[b][k] * P.nw[b];
        }
        // wall distribution on the line through the shifted and ghost points
        double fsp = d.fsp[0][(size_t)p * NV + k], gv = d.ghost[0][(size_t)p * NV + k];
        double fw = fsp + (gv - fsp) / (ygc - ysp) * (yw - ysp);
        acc[3] += d.w[k] * dn * dn * fw;
    }
    for (int b = 0; b < 4; ++b) {
        double s = block_sum(acc[b]);
        if (threadIdx.x == 0) d.pforce[4 * p + b] = b < 3 ? P.dS * s : s;
    }
}

// ---------------------------------------------------------------- state I/O
template <typename T>
__global__ void k_state_from_freestream(Dev d, int buf, int A, const double *u, double amp, long long off, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long long g = off + i;
    int k = (int)(g % d.NV);
    double v = d.fs[A][k] * (1.0 + (u ? amp * u[i] : 0.0));
    ((T *)d.f[buf][A])[g] = (T)v;
}

template <typename T>
__global__ void k_state_set(Dev d, int buf, int A, const double *src, long long off, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ((T *)d.f[buf][A])[off + i] = (T)src[i];
}

template <typename T>
__global__ void k_state_get(Dev d, int buf, int A, double *dst, long long off, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = (double)((const T *)d.f[buf][A])[off + i];
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

hipError_t launch_update(const Dev &d, int storage, int cur, int slot, hipStream_t s)
{
    long long waves = (long long)d.Nc * d.nchunk;
    DISPATCH(d.D, storage, hipLaunchKernelGGL((k_update<DD, TT>), dim3(blocks_for(waves, 4)), dim3(256), 0, s, d, cur, slot));
    return hipGetLastError();
}

hipError_t launch_update2d(const Dev &d, int storage, int cur, int slot, const Tile &t, hipStream_t s)
{
    const int W = 64 * t.V;
    const int ntx = (d.n[0] + t.TX - 1) / t.TX, nys = (d.n[1] + t.LY - 1) / t.LY, ncv = (d.NV + W - 1) / W;
    long long nblk = (long long)ntx * nys * ncv;
    nblk = (nblk + 7) / 8 * 8;
    dim3 grid((unsigned)nblk), block(64 * t.TX);
#define U2D(TT, VV, XX)                                                                                       \
    if (t.V == VV && t.TX == XX) {                                                                         \
        hipLaunchKernelGGL((k_update2d<TT, VV, XX>), grid, block, 0, s, d, cur, slot, t.LY, ntx, nys, ncv); \
        return hipGetLastError();                                                                          \
    }
    if (storage == 0) {
        U2D(double, 1, 4) U2D(double, 1, 8) U2D(double, 2, 4) U2D(double, 2, 8)
    } else {
        U2D(float, 1, 4) U2D(float, 1, 8) U2D(float, 2, 4) U2D(float, 2, 8) U2D(float, 4, 4) U2D(float, 4, 8)
    }
#undef U2D
    return hipErrorInvalidValue;
}

hipError_t launch_fill_fin(const Dev &d, int storage, int cur, int slot, bool fill, bool fin, hipStream_t s)
{
    int nfill = fill ? d.npairs : 0;
    int nfin = fin ? (int)blocks_for(d.Nc, 32) : 0;
    if (nfill + nfin == 0) return hipSuccess;
    DISPATCH(d.D, storage,
             hipLaunchKernelGGL((k_fill_fin<DD, TT>), dim3(nfill + nfin), dim3(256), 0, s, d, cur, slot, nfill, fin ? 1 : 0));
    return hipGetLastError();
}

hipError_t launch_moments_direct(const Dev &d, int storage, int cur, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, d.ctrl, slot);
    DISPATCH(d.D, storage, hipLaunchKernelGGL((k_moments_direct<DD, TT>), dim3(blocks_for(d.Nc, 4)), dim3(256), 0, s, d, cur, slot));
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
        hipLaunchKernelGGL(k_state_from_freestream<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, buf, A, u, amp, off, n);
    else
        hipLaunchKernelGGL(k_state_from_freestream<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, buf, A, u, amp, off, n);
    return hipGetLastError();
}

hipError_t launch_state_set(const Dev &d, int storage, int buf, int A, const double *src, long long off, long long n,
                            hipStream_t s)
{
    if (storage == 0)
        hipLaunchKernelGGL(k_state_set<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, buf, A, src, off, n);
    else
        hipLaunchKernelGGL(k_state_set<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, buf, A, src, off, n);
    return hipGetLastError();
}

hipError_t launch_state_get(const Dev &d, int storage, int buf, int A, double *dst, long long off, long long n,
                            hipStream_t s)
{
    if (storage == 0)
        hipLaunchKernelGGL(k_state_get<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, buf, A, dst, off, n);
    else
        hipLaunchKernelGGL(k_state_get<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, buf, A, dst, off, n);
    return hipGetLastError();
}

hipError_t launch_moments_out(const Dev &d, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments_out, dim3(blocks_for(d.Nc, 256)), dim3(256), 0, s, d, out);
    return hipGetLastError();
}

}  // namespace ibdvm
