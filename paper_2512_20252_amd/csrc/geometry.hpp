// geometry.hpp -- create-time preprocessing of the immersed boundary
// (arXiv 2512.20252, Section 3.2.1 cell and point classification, Section
// 3.2.2 surface cells, Section 3.2.3 velocity-space cut cells).  Host only;
// no HIP dependency, so a host-only context can be built without a device.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "device.hpp"

namespace ibdvm {

constexpr int kMaxSurface = 26;

enum VelClass : uint8_t { VC_GAS = 0, VC_SOLID = 1, VC_CUT_G = 2, VC_CUT_S = 3 };

struct Problem {
    int dim = 2;
    int n[3] = {1, 1, 1};
    double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
    int outer = 0;
    double lid_u = 0;
    int vn[3] = {1, 1, 1};
    double vlo[3] = {0, 0, 0}, vhi[3] = {0, 0, 0};
    int rule = 0;
    double vstretch = 0;
    double vref_amp = 0, vref_width = 1, vref_centre[3] = {0, 0, 0};  // refined rule
    int vweights = 0;  // 1: Jacobian weights of the mapped rules
    int gkind = 0;
    double gcen[3] = {0, 0, 0}, gsize[3] = {0, 0, 0}, aoa = 0;
    uint32_t flags = 0;
    double Uw[3] = {0, 0, 0}, Ow[3] = {0, 0, 0};  // body wall: translation and rotation about gcen
    bool moving_wall = false;
};

struct PairGeom {
    int gc, dc, ac, axis, sign, ns;
    int sc[kMaxSurface];
    int snb[kMaxSurface][3][2];  // fluid neighbours of each surface cell along each axis (-1: none)
    double xw[3], nw[3], xsp[3];
    double uw[3];  // wall velocity at x_w
    double r[kMaxSurface][3], rh[kMaxSurface][3];
};

struct Geometry {
    int D = 2, Nc = 0, NV = 0, nfluid = 0, nghost = 0;
    double dx[3] = {1, 1, 1};
    std::vector<double> xa[3], wa[3];  // per-axis velocity nodes and weights
    std::vector<double> ea0[3], ea1[3];  // per-axis dual cell [ea0, ea1] of each node
    double dxi[3] = {1, 1, 1};
    std::vector<double> xi;  // [NV*3]
    std::vector<double> w;   // [NV]
    std::vector<uint8_t> cflag;
    std::vector<int> pnb;  // [Nc*6]
    std::vector<PairGeom> pairs;
    std::vector<uint8_t> cls;  // [npairs*NV]
    std::vector<double> wg;    // [npairs*NV]
};

// 0 on success, else an ibdvm_status code with a message in err.
int build_geometry(const Problem &p, Geometry &g, std::string &err);

// measure of {v in box : n.v <= 0} (exposed for the closed-box identity tests)
double incident_measure(int dim, const double e0[3], const double e1[3], const double n[3]);

}  // namespace ibdvm
