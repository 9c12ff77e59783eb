// device.hpp -- layout of the tables the HIP kernels read (library-internal).
#pragma once
#include <cstdint>

namespace ibdvm {

// per-cell flags: solid; any stencil neighbour (+-1, +-2 along an axis) solid
// or outside the grid; and one bit per face neighbour that is solid
// (x-, x+, y-, y+, z-, z+)
enum CellFlag : uint8_t { CF_SOLID = 1, CF_NEAR = 2, CF_XM = 4, CF_XP = 8, CF_YM = 16, CF_YP = 32, CF_ZM = 64, CF_ZP = 128 };
// device flag words add: the cell two steps along -x / +x (-y / +y) is solid
constexpr int CF_XM2 = 256, CF_XP2 = 512, CF_YM2 = 1024, CF_YP2 = 2048;

// per-(cell, velocity chunk) partial moments of the new state, relative to
// the reference velocity U of the old state: m0, m1[D], m2, m3[D], M2[D(D+1)/2]
constexpr int kPartialWords2 = 9;
constexpr int kPartialWords3 = 14;
constexpr int kPartialStride = 16;
// per-cell parameter words: U[3], A, 1/T, s[3], T/2, 1/tau, rho, T, q[3], tau
constexpr int kCellWords = 16;
enum CellWord { CW_U = 0, CW_A = 3, CW_INVT = 4, CW_S = 5, CW_TH = 8, CW_INVTAU = 9, CW_RHO = 10, CW_T = 11, CW_Q = 12, CW_TAU = 15 };
// per-cell record of the marching updates, one contiguous 80-byte load.
// 2D: U0, U1, A, 1/T, s0, s1, T/2, 1/tau, then the flag word of the cell
// above (low half of word 8; 0 on the top row) and a pad word.  3D: U[3], A,
// 1/T, s[3], 1/tau, then the flag word of the cell above in z (word 9).
constexpr int kQWords = 10;

// convergence residual: conservative variables rho, rho U[3], rho E; per
// moment-finish workgroup the sums of squared changes, then of magnitudes
constexpr int kResVars = 5;
// cells per moment-finish workgroup: the explicit instance finishes four
// per wavefront (16 lanes each), the instance that can relax one per
// wavefront
constexpr int kFinCells = 16;
constexpr int kFinCellsRelax = 4;
// per pair: momentum flux through the face F[3], then at the wall point p_w,
// tau_w[3], q_n, and the raw moments of the wall distribution: sum w f,
// sum w xi f [3], sum w (|xi|^2 h + b) (3D: |xi|^2 f)
constexpr int kForceWords = 13;
// allocation-free surface forces: pairs the static force-record scratch holds
constexpr int kStaticMaxPairs = 16384;
// doubles per wall point in the device output of the allocation-free
// surface forces: x_w[3], n_w[3], rho_w, p_w, tau_w[3], q_n, C_p, T_s, u_s[3]
constexpr int kWallPointWords = 17;

// Dev::flags bits: semi-implicit collision (IBDVM_FLAG_IMPLICIT_COLLISION),
// face limit, naive extrapolation (IBDVM_FLAG_FACE_LIMIT,
// IBDVM_FLAG_NAIVE_EXTRAPOLATION)
constexpr unsigned kFlagImplicit = 1u << 2;
constexpr unsigned kFlagFaceLimit = 1u << 3;
constexpr unsigned kFlagNaive = 1u << 4;
// Dev::outer values
enum { kOuterFreestream = 0, kOuterPeriodic = 1, kOuterWalls = 2, kOuterSpecular = 3 };
constexpr int kChunk = 64;       // velocity nodes per wavefront
constexpr int kFillChunk = 256;  // velocity nodes per ghost-fill workgroup
constexpr int kMaxVn = 256;

struct DPair {
    int gc, dc, ac, axis, sign, ns;
    int sc[26];
    int snb[26][3][2];
    double ygc, ydc, yac, yw, ysp, yface;
    double den;  // sum over reflected measure of omega^s xi_n Hw
    double dS;   // face area
    double nw[3];
    double xw[3];  // intersect point
    double r[26][3];
    double rh[26][3];
};

struct Ctrl {
    unsigned long long tau_bits[2];
    double dt;
    double time;
    long long step;
    unsigned int health;
    unsigned int pad;
};

struct Dev {
    int D, NA, NV, nchunk, Nc, npairs, outer;
    unsigned flags;
    int n[3], vn[3];
    int stride[3], pad1;
    double dx[3], inv_dx[3];
    double adv, cfl, mu0, omega, Pr, Tw, alpha, shk;  // shk = 4(1-Pr)/5
    double Aw;                                         // wall Maxwellian prefactor (pi T_w)^(-D/2)
    const double *xi[3];
    const double *xa;  // per-axis nodes [3][kMaxVn]
    const double *w;
    const double *fs[2];
    const void *fsT[2];  // freestream rows in the storage type
    // 2D FP32 storage: reference the stored values are offsets from (the
    // freestream rows, or zeros); foff = 1 when it is the freestream
    const double *fr[2];
    int foff, pad2;
    const double *hw;
    const double *hwp;  // moving body wall: [pair][node] unit wall Maxwellian at the pair's wall velocity; else null
    void *f[2][2];  // [buffer][array]
    double *cellp;
    double *cellq;  // 2D: kQWords per cell
    double *part;
    const int *cflag;  // CellFlag bits per cell
    const int *pnb;
    const DPair *pairs;
    const uint8_t *cls;
    const double *wg;
    double *ghost[2], *face[2], *fiw[2], *fsp[2], *fwall[2];
    double *rhow;
    double *fillpart;  // [pair][fill chunk][2]: incident and specular partial wall fluxes
    double *pforce;
    double *respart;  // [moment-finish workgroup][2 kResVars]
    // outer walls (2D): ghost rows in the storage type, per array; rows
    // [0, ny) the wall x = lo (row j: cell (0, j)), [ny, 2ny) x = hi,
    // [2ny, 2ny + nx) y = lo (row 2ny + i: cell (i, 0)), then y = hi
    void *wallT[2];
    double lid_u;  // speed of the wall y = hi along +x
    // incoming normal flux sum_{xi_n < 0} w |xi_n| e^{-|xi - U_w|^2 / T_w} of
    // each outer wall (x = lo, x = hi, y = lo, y = hi)
    double wall_in[4];
    Ctrl *ctrl;
};

// argument block of a launch over several solves (serving form): solve s
// owns workgroups blk0[s] .. blk0[s+1]-1 of the launch; its parameter block
// is dev[s] (a copy of its Dev in its own workspace)
constexpr int kMaxBatch = 16;
struct BatchArgs {
    int n;
    int cur[kMaxBatch], slot[kMaxBatch];
    int LY[kMaxBatch], ntx[kMaxBatch], nys[kMaxBatch], ncv[kMaxBatch];
    int nfill[kMaxBatch];
    long long blk0[kMaxBatch + 1];
    const Dev *dev[kMaxBatch];
};

}  // namespace ibdvm
