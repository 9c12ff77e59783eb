// ibdvm.cpp -- C ABI of the immersed-boundary Shakhov-DVM library: context,
// workspace layout inside the caller's device buffer, table upload and the
// per-step launch sequence.  Declarations and argument conventions are in
// include/ibdvm.h.
#include "ibdvm.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "device.hpp"
#include "geometry.hpp"
#include "launch.hpp"

static_assert(ibdvm::kFlagImplicit == IBDVM_FLAG_IMPLICIT_COLLISION, "device flag bit of the semi-implicit collision");
static_assert(ibdvm::kFlagFaceLimit == IBDVM_FLAG_FACE_LIMIT, "device flag bit of the face limit");
static_assert(ibdvm::kFlagNaive == IBDVM_FLAG_NAIVE_EXTRAPOLATION, "device flag bit of the naive extrapolation");
static_assert((int)ibdvm::kOuterWalls == (int)IBDVM_OUTER_WALLS && (int)ibdvm::kOuterSpecular == (int)IBDVM_OUTER_SPECULAR &&
                  (int)ibdvm::kOuterPeriodic == (int)IBDVM_OUTER_PERIODIC, "device codes of the outer boundaries");

namespace {

thread_local std::string g_err;

ibdvm_status fail(ibdvm_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

constexpr double kPi = 3.14159265358979323846;

struct Layout {
    size_t f[2][2], cellp, cellq, part, xi, xa, w, fs, fsT, hw, cflag, pnb, pairs, cls, wg, ghost, face, fiw, fsp, fwall, rhow, fillpart, pforce, ctrl;
    size_t hwp;      // moving body wall: per pair the unit wall Maxwellian at its wall velocity
    size_t fr;       // 2D FP32 storage: the reference its values are offsets from
    size_t respart;  // moment-finish workgroups x 2 kResVars
    size_t wallT;    // outer walls: NA x 2(nx + ny) ghost rows in the storage type
    size_t devcopy;  // the context's Dev, read by launches over several solves
    size_t total;
    size_t state_bytes;  // one array of one buffer
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(const ibdvm::Geometry &g, int NA, int precision, const ibdvm::Problem &p)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t es = precision == IBDVM_F32_STORE ? 4 : 8;
    const size_t nf = (size_t)g.Nc * g.NV;
    const size_t np = g.pairs.size();
    const int nchunk = (g.NV + ibdvm::kChunk - 1) / ibdvm::kChunk;
    L.state_bytes = nf * es;
    for (int b = 0; b < 2; ++b)
        for (int A = 0; A < 2; ++A) L.f[b][A] = A < NA ? take(nf * es) : 0;
    L.cellp = take((size_t)g.Nc * ibdvm::kCellWords * 8);
    L.cellq = take((size_t)g.Nc * ibdvm::kQWords * 8);
    L.part = take((size_t)g.Nc * nchunk * ibdvm::kPartialStride * 8);
    L.xi = take((size_t)3 * g.NV * 8);
    L.xa = take((size_t)3 * ibdvm::kMaxVn * 8);
    L.w = take((size_t)g.NV * 8);
    L.fs = take((size_t)2 * g.NV * 8);
    L.fsT = take((size_t)2 * g.NV * es);
    L.fr = take((size_t)2 * g.NV * 8);
    L.hw = take((size_t)g.NV * 8);
    L.cflag = take((size_t)g.Nc * 4);
    L.pnb = take((size_t)g.Nc * 6 * 4);
    L.pairs = take(np * sizeof(ibdvm::DPair));
    L.cls = take(np * g.NV);
    L.wg = take(np * g.NV * 8);
    L.ghost = take((size_t)NA * np * g.NV * 8);
    L.face = take((size_t)NA * np * g.NV * 8);
    L.fiw = take((size_t)NA * np * g.NV * 8);
    L.fsp = take((size_t)NA * np * g.NV * 8);
    L.fwall = take((size_t)NA * np * g.NV * 8);
    L.rhow = take(np * 8);
    L.fillpart = take(np * ((g.NV + ibdvm::kFillChunk - 1) / ibdvm::kFillChunk) * 2 * 8);
    L.pforce = take(np * ibdvm::kForceWords * 8);
    L.respart = take((size_t)((g.Nc + ibdvm::kFinCellsRelax - 1) / ibdvm::kFinCellsRelax) * 2 * ibdvm::kResVars * 8);
    L.wallT = take(p.outer == IBDVM_OUTER_WALLS || p.outer == IBDVM_OUTER_SPECULAR
                       ? (size_t)NA * 2 * (p.n[0] + p.n[1]) * g.NV * es
                       : 0);
    L.hwp = take(p.moving_wall ? np * g.NV * 8 : 0);
    L.ctrl = take(sizeof(ibdvm::Ctrl));
    L.devcopy = take(sizeof(ibdvm::Dev));
    L.total = off;
    return L;
}

ibdvm_status validate(const ibdvm_grid *grid, const ibdvm_vgrid *vg, const ibdvm_geometry *geom, const ibdvm_opts *opts,
                      ibdvm::Problem &p)
{
    if (!grid || !vg || !geom || !opts) return fail(IBDVM_E_INVALID_ARG, "null argument");
    if (grid->dim != 2 && grid->dim != 3) return fail(IBDVM_E_INVALID_ARG, "dim must be 2 or 3");
    p = ibdvm::Problem{};
    p.dim = grid->dim;
    for (int a = 0; a < 3; ++a) {
        bool used = a < grid->dim;
        p.n[a] = used ? grid->n[a] : 1;
        p.lo[a] = used ? grid->lo[a] : 0.0;
        p.hi[a] = used ? grid->hi[a] : 1.0;
        p.vn[a] = used ? vg->n[a] : 1;
        p.vlo[a] = used ? vg->lo[a] : 0.0;
        p.vhi[a] = used ? vg->hi[a] : 0.0;
        p.gcen[a] = geom->center[a];
        p.gsize[a] = geom->size[a];
        if (!used) continue;
        if (grid->n[a] < 4) return fail(IBDVM_E_INVALID_ARG, "grid needs at least 4 cells per axis");
        if (!(grid->hi[a] > grid->lo[a])) return fail(IBDVM_E_INVALID_ARG, "grid box is empty");
        if (vg->n[a] < 2 || vg->n[a] > ibdvm::kMaxVn) return fail(IBDVM_E_INVALID_ARG, "velocity nodes per axis must be in [2, 256]");
        if (!(vg->hi[a] > 0.0) || vg->lo[a] != -vg->hi[a])
            return fail(IBDVM_E_INVALID_ARG, "velocity box must be symmetric about 0");
    }
    if (grid->outer_bc != IBDVM_OUTER_FREESTREAM && grid->outer_bc != IBDVM_OUTER_PERIODIC &&
        grid->outer_bc != IBDVM_OUTER_WALLS && grid->outer_bc != IBDVM_OUTER_SPECULAR)
        return fail(IBDVM_E_INVALID_ARG, "unknown outer boundary condition");
    if ((grid->outer_bc == IBDVM_OUTER_WALLS || grid->outer_bc == IBDVM_OUTER_SPECULAR) && grid->dim != 2)
        return fail(IBDVM_E_UNSUPPORTED, "outer walls are implemented for dim 2 only");
    if (grid->outer_bc == IBDVM_OUTER_WALLS && !std::isfinite(grid->lid_u))
        return fail(IBDVM_E_INVALID_ARG, "lid speed must be finite");
    p.outer = grid->outer_bc;
    p.lid_u = grid->outer_bc == IBDVM_OUTER_WALLS ? grid->lid_u : 0.0;
    if (vg->rule != IBDVM_RULE_MIDPOINT && vg->rule != IBDVM_RULE_TRAPEZOID && vg->rule != IBDVM_RULE_STRETCHED &&
        vg->rule != IBDVM_RULE_REFINED)
        return fail(IBDVM_E_INVALID_ARG, "unknown quadrature rule");
    if (vg->rule == IBDVM_RULE_REFINED) {
        if (!(vg->refine_amp >= 0.0 && std::isfinite(vg->refine_amp)) ||
            !(vg->refine_width > 0.0 && std::isfinite(vg->refine_width)))
            return fail(IBDVM_E_INVALID_ARG, "refinement amplitude must be >= 0 and width > 0");
        for (int a = 0; a < grid->dim; ++a) {
            if (!(std::fabs(vg->refine_centre[a]) < vg->hi[a]))
                return fail(IBDVM_E_INVALID_ARG, "refinement centre must lie inside the velocity box");
            if (grid->outer_bc == IBDVM_OUTER_SPECULAR && vg->refine_centre[a] != 0.0)
                return fail(IBDVM_E_INVALID_ARG, "specular walls need nodes symmetric about 0 (refinement centre 0)");
            p.vref_centre[a] = vg->refine_centre[a];
        }
        p.vref_amp = vg->refine_amp;
        p.vref_width = vg->refine_width;
    }
    if (vg->rule == IBDVM_RULE_STRETCHED && !(vg->stretch > 0.0 && vg->stretch <= 20.0))
        return fail(IBDVM_E_INVALID_ARG, "stretch must be in (0, 20]");
    p.rule = vg->rule;
    p.vstretch = vg->rule == IBDVM_RULE_STRETCHED ? vg->stretch : 0.0;
    if (vg->weights != IBDVM_WEIGHTS_CELL &&
        !(vg->weights == IBDVM_WEIGHTS_JACOBIAN && (vg->rule == IBDVM_RULE_STRETCHED || vg->rule == IBDVM_RULE_REFINED)))
        return fail(IBDVM_E_INVALID_ARG, "Jacobian weights need a stretched or refined velocity grid");
    p.vweights = vg->weights;
    int k = geom->kind;
    bool ok2 = k == IBDVM_GEOM_NONE || k == IBDVM_GEOM_CIRCLE || k == IBDVM_GEOM_ELLIPSE || k == IBDVM_GEOM_AIRFOIL;
    bool ok3 = k == IBDVM_GEOM_NONE || k == IBDVM_GEOM_SPHERE;
    if ((grid->dim == 2 && !ok2) || (grid->dim == 3 && !ok3)) return fail(IBDVM_E_INVALID_ARG, "geometry kind does not match dim");
    if (k != IBDVM_GEOM_NONE && !(geom->size[0] > 0.0)) return fail(IBDVM_E_INVALID_ARG, "geometry size must be positive");
    if ((k == IBDVM_GEOM_ELLIPSE || k == IBDVM_GEOM_AIRFOIL) && !(geom->size[1] > 0.0))
        return fail(IBDVM_E_INVALID_ARG, "geometry size[1] must be positive");
    p.gkind = k;
    p.aoa = geom->aoa_rad;
    p.flags = opts->flags;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(opts->U_w[a]) || !std::isfinite(opts->Omega_w[a]))
            return fail(IBDVM_E_INVALID_ARG, "wall velocity must be finite");
        p.Uw[a] = opts->U_w[a];
        p.Ow[a] = opts->Omega_w[a];
        if (p.Uw[a] != 0.0 || p.Ow[a] != 0.0) p.moving_wall = k != IBDVM_GEOM_NONE;
    }
    if (opts->precision != IBDVM_F64 && opts->precision != IBDVM_F32_STORE) return fail(IBDVM_E_INVALID_ARG, "unknown precision");
    if (!(opts->cfl > 0.0 && opts->cfl <= 1.0)) return fail(IBDVM_E_INVALID_ARG, "cfl must be in (0, 1]");
    if (!(opts->omega_vhs > 0.0 && opts->omega_vhs < 2.5) || !(opts->a_vhs > 0.0))
        return fail(IBDVM_E_INVALID_ARG, "viscosity law parameters out of range");
    return IBDVM_OK;
}

#define HIP_CHECK(expr)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(IBDVM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

struct ibdvm_ctx {
    ibdvm::Problem prob;
    ibdvm::Geometry geo;
    double Kn = 0, Ma = 0, Pr = 0, gam = 0, alpha = 1, Tw = 1, cfl = 0.5, omega = 0.81, avhs = 1.0;
    int precision = 0;
    int NA = 2;
    bool host_only = false;
    bool broken = false;
    int device = 0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    Layout L{};
    ibdvm::Dev dev{};
    int cur = 0;
    long long step = 0;
    bool pending = false;
    int fin_cells = ibdvm::kFinCells;  // cells per workgroup of the last moment finish (its residual partials)
    bool res_valid = false;  // a step has run since the state was set: residual partials hold its change
    double Uinf = 0, mu0 = 0, Lref = 1;
    ibdvm::Tile tile{1, 8, 64};
    bool profiling = false;
    std::vector<hipEvent_t> ev[2];  // start/stop pairs per kernel kind
    ~ibdvm_ctx()
    {
        for (auto &v : ev)
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
    }
};

namespace {

ibdvm_status sync_and_check(ibdvm_ctx *c)
{
    HIP_CHECK(hipStreamSynchronize(c->stream));
    unsigned health = 0;
    HIP_CHECK(hipMemcpy(&health, c->ws + c->L.ctrl + offsetof(ibdvm::Ctrl, health), sizeof(health), hipMemcpyDeviceToHost));
    if (health) {
        c->broken = true;
        return fail(IBDVM_E_UNSTABLE, "non-physical state (NaN, rho <= 0 or T <= 0)");
    }
    return IBDVM_OK;
}

ibdvm_status require_device(const ibdvm_ctx *c)
{
    if (!c) return fail(IBDVM_E_INVALID_ARG, "null context");
    if (c->host_only) return fail(IBDVM_E_STATE, "host-only context has no device state");
    if (c->broken) return fail(IBDVM_E_STATE, "context became unstable; destroy it");
    return IBDVM_OK;
}

// moments of the current state by direct summation, tau_min into its slot
ibdvm_status refresh_moments(ibdvm_ctx *c)
{
    HIP_CHECK(ibdvm::launch_moments_direct(c->dev, c->precision, c->cur, (int)(c->step & 1), c->stream));
    c->pending = false;
    c->res_valid = false;
    return IBDVM_OK;
}

ibdvm_status reset_clock(ibdvm_ctx *c)
{
    ibdvm::Ctrl ctrl{};
    ctrl.tau_bits[0] = ctrl.tau_bits[1] = 0x7ff0000000000000ull;
    HIP_CHECK(hipMemcpyAsync(c->ws + c->L.ctrl, &ctrl, sizeof(ctrl), hipMemcpyHostToDevice, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    c->step = 0;
    c->cur = 0;
    return IBDVM_OK;
}

// moves host arrays [cells][nodes] into buffer `cur` in chunks staged through
// the other buffer (free while the state is being replaced)
ibdvm_status upload_state(ibdvm_ctx *c, const double *src[2], const double *noise[2], double amp)
{
    const long long NV = c->geo.NV, Nc = c->geo.Nc;
    const int other = c->cur ^ 1;
    char *stage = c->ws + c->L.f[other][0];
    size_t stage_bytes = c->L.state_bytes * c->NA;
    long long chunk_cells = std::max<long long>(1, (long long)(stage_bytes / (NV * 8)));
    for (int A = 0; A < c->NA; ++A) {
        for (long long c0 = 0; c0 < Nc; c0 += chunk_cells) {
            long long nc = std::min(chunk_cells, Nc - c0);
            long long n = nc * NV, off = c0 * NV;
            const double *h = src ? src[A] : noise[A];
            if (h) {
                HIP_CHECK(hipMemcpyAsync(stage, h + off, n * 8, hipMemcpyHostToDevice, c->stream));
            }
            if (src)
                HIP_CHECK(ibdvm::launch_state_set(c->dev, c->precision, c->cur, A, (const double *)stage, off, n, c->stream));
            else
                HIP_CHECK(ibdvm::launch_state_freestream(c->dev, c->precision, c->cur, A, h ? (const double *)stage : nullptr,
                                                          amp, off, n, c->stream));
            HIP_CHECK(hipStreamSynchronize(c->stream));
        }
    }
    return IBDVM_OK;
}

ibdvm_status mark(ibdvm_ctx *c, int kind)
{
    if (!c->profiling) return IBDVM_OK;
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    HIP_CHECK(hipEventRecord(e, c->stream));
    c->ev[kind].push_back(e);
    return IBDVM_OK;
}

// the device copy of the context's Dev (launches over several solves read it)
ibdvm_status put_dev(ibdvm_ctx *c)
{
    HIP_CHECK(hipMemcpyAsync(c->ws + c->L.devcopy, &c->dev, sizeof(c->dev), hipMemcpyHostToDevice, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    return IBDVM_OK;
}

// cells per workgroup of the finish instance a context's own launches take
int own_fin_cells(const ibdvm_ctx *c)
{
    return (c->prob.flags & IBDVM_FLAG_IMPLICIT_COLLISION) ? ibdvm::kFinCellsRelax : ibdvm::kFinCells;
}

ibdvm_status one_step(ibdvm_ctx *c)
{
    const int slot = (int)(c->step & 1);
    ibdvm_status st;
    if ((st = mark(c, 1))) return st;
    if (c->pending && (c->prob.flags & IBDVM_FLAG_IMPLICIT_COLLISION)) {
        // the moment finish relaxes the state, so it completes before the
        // ghost fill reads it
        HIP_CHECK(ibdvm::launch_fill_fin(c->dev, c->precision, c->cur, slot, false, true, c->stream));
        c->pending = false;
        c->fin_cells = own_fin_cells(c);
    }
    if (c->pending) c->fin_cells = own_fin_cells(c);
    HIP_CHECK(ibdvm::launch_fill_fin(c->dev, c->precision, c->cur, slot, true, c->pending, c->stream));
    HIP_CHECK(ibdvm::launch_wall_fill(c->dev, c->precision, c->cur, c->stream));
    if ((st = mark(c, 1)) || (st = mark(c, 0))) return st;
    if (c->prob.dim == 2)
        HIP_CHECK(ibdvm::launch_update2d(c->dev, c->precision, c->cur, slot, c->tile, c->stream));
    else
        HIP_CHECK(ibdvm::launch_update3d(c->dev, c->precision, c->cur, slot, c->tile, c->stream));
    if ((st = mark(c, 0))) return st;
    c->cur ^= 1;
    c->step += 1;
    c->pending = true;
    c->res_valid = true;
    return IBDVM_OK;
}

ibdvm_status finish_pending(ibdvm_ctx *c)
{
    if (!c->pending) return IBDVM_OK;
    HIP_CHECK(ibdvm::launch_fill_fin(c->dev, c->precision, c->cur, (int)(c->step & 1), false, true, c->stream));
    c->pending = false;
    c->fin_cells = own_fin_cells(c);
    return IBDVM_OK;
}

// ---- launches over several contexts that share one stream (serving form).
// Every fill phase is one launch per (dimension, storage) group and the 2D
// update one launch per (storage, V, TX) group, each over the workgroups of
// all the group's solves (at most kMaxBatch per launch); the 3D update is
// launched per context.  Each solve's arithmetic is that of one_step.

void batch_entry(ibdvm::BatchArgs &a, int q, const ibdvm_ctx *c)
{
    a.dev[q] = (const ibdvm::Dev *)(c->ws + c->L.devcopy);
    a.cur[q] = c->cur;
    a.slot[q] = (int)(c->step & 1);
}

// the fill phases (fill) and the moment finish of pending contexts
ibdvm_status fused_fill(ibdvm_ctx *const *cs, int n, bool fill, hipStream_t stream)
{
    if (fill) {
        // a semi-implicit solve relaxes in its moment finish: finish first
        bool split = false;
        for (int i = 0; i < n; ++i) split = split || (cs[i]->pending && (cs[i]->prob.flags & IBDVM_FLAG_IMPLICIT_COLLISION));
        if (split) {
            ibdvm_status st = fused_fill(cs, n, false, stream);
            if (st) return st;
        }
    }
    for (int D = 2; D <= 3; ++D)
        for (int prec = 0; prec < 2; ++prec) {
            std::vector<ibdvm_ctx *> grp;
            for (int i = 0; i < n; ++i)
                if (cs[i]->prob.dim == D && cs[i]->precision == prec) grp.push_back(cs[i]);
            for (size_t b = 0; b < grp.size(); b += ibdvm::kMaxBatch) {
                const int m = (int)std::min<size_t>(ibdvm::kMaxBatch, grp.size() - b);
                ibdvm::BatchArgs fin{}, spec{}, ghost{};
                fin.n = spec.n = ghost.n = m;
                bool implicit = false;
                for (int q = 0; q < m; ++q)
                    implicit = implicit || (grp[b + q]->pending && (grp[b + q]->prob.flags & IBDVM_FLAG_IMPLICIT_COLLISION));
                // one finish instance serves the batch: the one that can relax if any member needs it
                const int cpb = implicit ? ibdvm::kFinCellsRelax : ibdvm::kFinCells;
                for (int q = 0; q < m; ++q) {
                    ibdvm_ctx *c = grp[b + q];
                    const int nfc = (c->geo.NV + ibdvm::kFillChunk - 1) / ibdvm::kFillChunk;
                    const int nfill = fill ? c->dev.npairs * nfc : 0;
                    const int nfin = c->pending ? (c->geo.Nc + cpb - 1) / cpb : 0;
                    if (c->pending) c->fin_cells = cpb;
                    for (ibdvm::BatchArgs *a : {&fin, &spec, &ghost}) {
                        batch_entry(*a, q, c);
                        a->nfill[q] = nfill;
                    }
                    fin.blk0[q + 1] = fin.blk0[q] + nfill + nfin;
                    spec.blk0[q + 1] = spec.blk0[q] + (c->dev.alpha < 1.0 ? nfill : 0);
                    ghost.blk0[q + 1] = ghost.blk0[q] + nfill;
                }
                HIP_CHECK(ibdvm::launch_fill_batch(D, prec, fin, spec, ghost, implicit, stream));
            }
        }
    for (int i = 0; i < n; ++i) cs[i]->pending = false;
    return IBDVM_OK;
}

ibdvm_status fused_step(ibdvm_ctx *const *cs, int n, hipStream_t stream)
{
    ibdvm_status st = fused_fill(cs, n, true, stream);
    if (st) return st;
    for (int i = 0; i < n; ++i) HIP_CHECK(ibdvm::launch_wall_fill(cs[i]->dev, cs[i]->precision, cs[i]->cur, stream));
    for (int walls = 0; walls < 2; ++walls)
        for (int prec = 0; prec < 2; ++prec)
            for (int V = 1; V <= 2; ++V)
                for (int TX = 4; TX <= 8; TX += 4) {
                    std::vector<ibdvm_ctx *> grp;
                    for (int i = 0; i < n; ++i) {
                        const ibdvm_ctx *c = cs[i];
                        if (c->prob.dim == 2 && c->precision == prec && c->tile.V == V && c->tile.TX == TX &&
                            (c->prob.outer == IBDVM_OUTER_WALLS || c->prob.outer == IBDVM_OUTER_SPECULAR) == (walls == 1))
                            grp.push_back(cs[i]);
                    }
                    for (size_t b = 0; b < grp.size(); b += ibdvm::kMaxBatch) {
                        const int m = (int)std::min<size_t>(ibdvm::kMaxBatch, grp.size() - b);
                        ibdvm::BatchArgs a{};
                        a.n = m;
                        for (int q = 0; q < m; ++q) {
                            const ibdvm_ctx *c = grp[b + q];
                            batch_entry(a, q, c);
                            a.LY[q] = c->tile.LY;
                            a.ntx[q] = (c->prob.n[0] + TX - 1) / TX;
                            a.nys[q] = (c->prob.n[1] + c->tile.LY - 1) / c->tile.LY;
                            a.ncv[q] = (c->geo.NV + 64 * V - 1) / (64 * V);
                            a.blk0[q + 1] = a.blk0[q] + (long long)a.ntx[q] * a.nys[q] * a.ncv[q];
                        }
                        HIP_CHECK(ibdvm::launch_update2d_batch(prec, V, TX, walls == 1, a, stream));
                    }
                }
    for (int i = 0; i < n; ++i) {
        ibdvm_ctx *c = cs[i];
        if (c->prob.dim == 3)
            HIP_CHECK(ibdvm::launch_update3d(c->dev, c->precision, c->cur, (int)(c->step & 1), c->tile, stream));
        c->cur ^= 1;
        c->step += 1;
        c->pending = true;
        c->res_valid = true;
    }
    return IBDVM_OK;
}

ibdvm_status check_batch(ibdvm_ctx *const *ctxs, int32_t n)
{
    if (!ctxs || n < 0) return fail(IBDVM_E_INVALID_ARG, "bad batch arguments");
    for (int32_t i = 0; i < n; ++i) {
        ibdvm_status st = require_device(ctxs[i]);
        if (st) return st;
        if (ctxs[i]->stream != ctxs[0]->stream || ctxs[i]->device != ctxs[0]->device)
            return fail(IBDVM_E_INVALID_ARG, "batched contexts must share one stream and device");
        for (int32_t j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(IBDVM_E_INVALID_ARG, "a context appears twice in the batch");
    }
    return IBDVM_OK;
}

ibdvm_status build(const ibdvm_grid *grid, const ibdvm_vgrid *vg, const ibdvm_geometry *geom, const ibdvm_opts *opts,
                   ibdvm_ctx &c)
{
    ibdvm_status st = validate(grid, vg, geom, opts, c.prob);
    if (st) return st;
    std::string err;
    int code = ibdvm::build_geometry(c.prob, c.geo, err);
    if (code) return fail((ibdvm_status)code, err);
    c.NA = c.prob.dim == 2 ? 2 : 1;
    c.precision = opts->precision;
    c.L = make_layout(c.geo, c.NA, c.precision, c.prob);
    return IBDVM_OK;
}

}  // namespace

extern "C" {

const char *ibdvm_last_error(void) { return g_err.c_str(); }

ibdvm_status ibdvm_footprint(const ibdvm_grid *grid, const ibdvm_vgrid *vgrid, const ibdvm_geometry *geom,
                             const ibdvm_opts *opts, size_t *bytes)
{
    if (!bytes) return fail(IBDVM_E_INVALID_ARG, "null output");
    ibdvm_ctx c;
    ibdvm_status st = build(grid, vgrid, geom, opts, c);
    if (st) return st;
    *bytes = c.L.total;
    return IBDVM_OK;
}

ibdvm_status ibdvm_create(const ibdvm_grid *grid, const ibdvm_vgrid *vgrid, const ibdvm_geometry *geom, double Kn,
                          double Ma, double Pr, double gamma, double alpha, double T_w, const ibdvm_opts *opts,
                          ibdvm_ctx **out)
{
    if (!out) return fail(IBDVM_E_INVALID_ARG, "null output");
    *out = nullptr;
    if (!(Kn > 0.0) || !(Ma >= 0.0) || !(Pr > 0.0) || !(gamma > 1.0) || !(alpha >= 0.0 && alpha <= 1.0) || !(T_w > 0.0))
        return fail(IBDVM_E_INVALID_ARG, "physical parameter out of range");
    ibdvm_ctx *c = new ibdvm_ctx();
    ibdvm_status st = build(grid, vgrid, geom, opts, *c);
    if (st) {
        delete c;
        return st;
    }
    c->Kn = Kn;
    c->Ma = Ma;
    c->Pr = Pr;
    c->gam = gamma;
    c->alpha = alpha;
    c->Tw = T_w;
    c->cfl = opts->cfl;
    c->omega = opts->omega_vhs;
    c->avhs = opts->a_vhs;
    c->host_only = (opts->flags & IBDVM_FLAG_HOST_ONLY) != 0;
    const double al = c->avhs, om = c->omega;
    c->mu0 = 5.0 * (al + 1.0) * (al + 2.0) * std::sqrt(kPi) / (4.0 * al * (5.0 - 2.0 * om) * (7.0 - 2.0 * om)) * Kn;
    c->Uinf = Ma * std::sqrt(gamma / 2.0);
    switch (c->prob.gkind) {
    case IBDVM_GEOM_CIRCLE:
    case IBDVM_GEOM_ELLIPSE:
        c->Lref = 2.0 * c->prob.gsize[0];
        break;
    case IBDVM_GEOM_AIRFOIL:
        c->Lref = c->prob.gsize[0];
        break;
    case IBDVM_GEOM_SPHERE:
        c->Lref = kPi * c->prob.gsize[0] * c->prob.gsize[0];
        break;
    default:
        c->Lref = 1.0;
    }
    if (c->host_only) {
        *out = c;
        return IBDVM_OK;
    }
    if (!opts->workspace) {
        delete c;
        return fail(IBDVM_E_INVALID_ARG, "workspace is NULL");
    }
    if (((uintptr_t)opts->workspace & 255u) != 0) {
        delete c;
        return fail(IBDVM_E_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    if (opts->workspace_bytes < c->L.total) {
        size_t need = c->L.total;
        delete c;
        return fail(IBDVM_E_NO_MEMORY, "workspace smaller than footprint (" + std::to_string(need) + " bytes)");
    }
    c->ws = (char *)opts->workspace;
    c->stream = (hipStream_t)opts->stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(IBDVM_E_DEVICE, "no HIP device");
    }

    // host tables
    const ibdvm::Geometry &g = c->geo;
    const int D = c->prob.dim, NV = g.NV;
    const size_t np = g.pairs.size();
    std::vector<double> xi((size_t)3 * NV, 0.0), xa((size_t)3 * ibdvm::kMaxVn, 0.0), fs((size_t)2 * NV, 0.0), hw(NV);
    double adv = 0.0;
    for (int a = 0; a < D; ++a) {
        double mx = 0.0;
        for (int i = 0; i < c->prob.vn[a]; ++i) {
            xa[(size_t)a * ibdvm::kMaxVn + i] = g.xa[a][i];
            mx = std::max(mx, std::fabs(g.xa[a][i]));
        }
        adv += mx / g.dx[a];
    }
    const double Aw = D == 2 ? 1.0 / (kPi * T_w) : std::pow(kPi * T_w, -1.5);
    const double Af = D == 2 ? 1.0 / kPi : std::pow(kPi, -1.5);
    for (int k = 0; k < NV; ++k) {
        double x2 = 0.0, c2 = 0.0;
        for (int a = 0; a < D; ++a) {
            double x = g.xi[3 * k + a];
            xi[(size_t)a * NV + k] = x;
            x2 += x * x;
            double cc = x - (a == 0 ? c->Uinf : 0.0);
            c2 += cc * cc;
        }
        hw[k] = Aw * std::exp(-x2 / T_w);
        fs[k] = Af * std::exp(-c2);
        fs[(size_t)NV + k] = 0.5 * fs[k];
    }
    // moving body wall: the unit wall Maxwellian of each pair at its wall velocity
    std::vector<double> hwp(c->prob.moving_wall ? np * NV : 0);
    for (size_t ip = 0; ip < np && c->prob.moving_wall; ++ip)
        for (int k = 0; k < NV; ++k) {
            double c2 = 0.0;
            for (int a = 0; a < D; ++a) {
                const double cc = g.xi[3 * k + a] - g.pairs[ip].uw[a];
                c2 += cc * cc;
            }
            hwp[ip * NV + k] = Aw * std::exp(-c2 / T_w);
        }
    std::vector<ibdvm::DPair> dp(np);
    for (size_t ip = 0; ip < np; ++ip) {
        const ibdvm::PairGeom &p = g.pairs[ip];
        ibdvm::DPair &q = dp[ip];
        std::memset(&q, 0, sizeof(q));
        q.gc = p.gc;
        q.dc = p.dc;
        q.ac = p.ac;
        q.axis = p.axis;
        q.sign = p.sign;
        q.ns = p.ns;
        const int a = p.axis;
        int ig = p.gc, ia[3];
        ia[0] = ig % c->prob.n[0];
        ia[1] = (ig / c->prob.n[0]) % c->prob.n[1];
        ia[2] = D == 3 ? ig / (c->prob.n[0] * c->prob.n[1]) : 0;
        auto centre = [&](int i) { return c->prob.lo[a] + ((double)i + 0.5) * g.dx[a]; };
        q.ygc = centre(ia[a]);
        q.ydc = centre(ia[a] + p.sign);
        q.yac = p.ac >= 0 ? centre(ia[a] + 2 * p.sign) : 0.0;
        q.yw = p.xw[a];
        q.ysp = p.xsp[a];
        q.yface = q.ygc + 0.5 * p.sign * g.dx[a];
        q.dS = 1.0;
        for (int b = 0; b < D; ++b)
            if (b != a) q.dS *= g.dx[b];
        for (int b = 0; b < 3; ++b) {
            q.nw[b] = p.nw[b];
            q.xw[b] = p.xw[b];
        }
        for (int j = 0; j < p.ns; ++j) {
            q.sc[j] = p.sc[j];
            for (int b = 0; b < 3; ++b) {
                q.r[j][b] = p.r[j][b];
                q.rh[j][b] = p.rh[j][b];
                q.snb[j][b][0] = p.snb[j][b][0];
                q.snb[j][b][1] = p.snb[j][b][1];
            }
        }
        double den = 0.0;
        for (int k = 0; k < NV; ++k) {
            uint8_t cl = g.cls[ip * NV + k];
            double ws = cl == ibdvm::VC_SOLID ? g.w[k] : (cl >= 2 ? g.w[k] - g.wg[ip * NV + k] : 0.0);
            double dn = 0.0;
            for (int b = 0; b < D; ++b) dn += g.xi[3 * k + b] * p.nw[b];
            den += ws * dn * (c->prob.moving_wall ? hwp[ip * NV + k] : hw[k]);
        }
        q.den = den;
    }

    // device view
    ibdvm::Dev &d = c->dev;
    std::memset(&d, 0, sizeof(d));
    d.D = D;
    d.NA = c->NA;
    d.NV = NV;
    if (D == 2)
        c->tile = c->precision == IBDVM_F32_STORE ? ibdvm::Tile{2, 8, 64} : ibdvm::Tile{1, 8, 64};
    else
        c->tile = ibdvm::Tile{1, 16, 256};
    d.nchunk = (NV + 64 * c->tile.V - 1) / (64 * c->tile.V);
    d.Nc = g.Nc;
    d.npairs = (int)np;
    d.outer = c->prob.outer;
    d.lid_u = c->prob.lid_u;
    if (c->prob.outer == IBDVM_OUTER_WALLS)
        for (int a = 0; a < 2; ++a)
            for (int sd = 0; sd < 2; ++sd) {
                const double Ux = (a == 1 && sd == 1) ? c->prob.lid_u : 0.0, side = sd ? 1.0 : -1.0;
                double in = 0.0;
                for (int k = 0; k < NV; ++k) {
                    const double xn = side * g.xi[3 * k + a];
                    if (xn < 0.0) {
                        const double cx = g.xi[3 * k] - Ux, cy = g.xi[3 * k + 1];
                        in -= g.w[k] * xn * std::exp(-(cx * cx + cy * cy) / T_w);
                    }
                }
                d.wall_in[2 * a + sd] = in;
            }
    d.flags = c->prob.flags;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = c->prob.n[a];
        d.vn[a] = c->prob.vn[a];
        d.dx[a] = g.dx[a];
        d.inv_dx[a] = 1.0 / g.dx[a];
    }
    d.stride[0] = 1;
    d.stride[1] = c->prob.n[0];
    d.stride[2] = c->prob.n[0] * c->prob.n[1];
    d.adv = adv;
    d.cfl = c->cfl;
    d.mu0 = c->mu0;
    d.omega = c->omega;
    d.Pr = Pr;
    d.Tw = T_w;
    d.alpha = alpha;
    d.shk = 4.0 * (1.0 - Pr) / 5.0;
    d.Aw = Aw;
    char *ws = c->ws;
    const Layout &L = c->L;
    for (int a = 0; a < 3; ++a) d.xi[a] = (const double *)(ws + L.xi) + (size_t)a * NV;
    d.xa = (const double *)(ws + L.xa);
    d.w = (const double *)(ws + L.w);
    d.fs[0] = (const double *)(ws + L.fs);
    d.fs[1] = (const double *)(ws + L.fs) + NV;
    d.hw = (const double *)(ws + L.hw);
    d.hwp = c->prob.moving_wall ? (const double *)(ws + L.hwp) : nullptr;
    // 2D FP32 storage keeps offsets from the freestream unless asked for f itself
    d.foff = (D == 2 && c->precision == IBDVM_F32_STORE && !(c->prob.flags & IBDVM_FLAG_F32_ABSOLUTE)) ? 1 : 0;
    d.fr[0] = (const double *)(ws + L.fr);
    d.fr[1] = (const double *)(ws + L.fr) + NV;
    d.fsT[0] = ws + L.fsT;
    d.fsT[1] = ws + L.fsT + (c->precision == IBDVM_F32_STORE ? 4 : 8) * (size_t)NV;
    for (int b = 0; b < 2; ++b)
        for (int A = 0; A < 2; ++A) d.f[b][A] = A < c->NA ? (void *)(ws + L.f[b][A]) : nullptr;
    d.cellp = (double *)(ws + L.cellp);
    d.cellq = (double *)(ws + L.cellq);
    d.part = (double *)(ws + L.part);
    d.cflag = (const int *)(ws + L.cflag);
    d.pnb = (const int *)(ws + L.pnb);
    d.pairs = (const ibdvm::DPair *)(ws + L.pairs);
    d.cls = (const uint8_t *)(ws + L.cls);
    d.wg = (const double *)(ws + L.wg);
    const size_t pstride = np * NV;
    for (int A = 0; A < 2; ++A) {
        int AA = A < c->NA ? A : 0;
        d.ghost[A] = (double *)(ws + L.ghost) + AA * pstride;
        d.face[A] = (double *)(ws + L.face) + AA * pstride;
        d.fiw[A] = (double *)(ws + L.fiw) + AA * pstride;
        d.fsp[A] = (double *)(ws + L.fsp) + AA * pstride;
        d.fwall[A] = (double *)(ws + L.fwall) + AA * pstride;
    }
    d.rhow = (double *)(ws + L.rhow);
    d.fillpart = (double *)(ws + L.fillpart);
    d.pforce = (double *)(ws + L.pforce);
    d.respart = (double *)(ws + L.respart);
    {
        const size_t wrow = (size_t)2 * (c->prob.n[0] + c->prob.n[1]) * NV * (c->precision == IBDVM_F32_STORE ? 4 : 8);
        for (int A = 0; A < 2; ++A)
            d.wallT[A] = c->prob.outer == IBDVM_OUTER_WALLS || c->prob.outer == IBDVM_OUTER_SPECULAR
                             ? (void *)(ws + L.wallT + (A < c->NA ? A : 0) * wrow)
                             : nullptr;
    }
    d.ctrl = (ibdvm::Ctrl *)(ws + L.ctrl);

    auto up = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(L.xi, xi.data(), xi.size() * 8);
    if (e == hipSuccess) e = up(L.xa, xa.data(), xa.size() * 8);
    if (e == hipSuccess) e = up(L.w, g.w.data(), g.w.size() * 8);
    if (e == hipSuccess) e = up(L.fs, fs.data(), fs.size() * 8);
    if (e == hipSuccess) e = up(L.hw, hw.data(), hw.size() * 8);
    if (e == hipSuccess) e = up(L.hwp, hwp.data(), hwp.size() * 8);
    // the freestream rows in the storage type: 2D FP32 storage holds offsets
    // from the freestream, so its freestream rows are zero
    std::vector<float> fs32(fs.size(), 0.0f);
    if (!d.foff) fs32.assign(fs.begin(), fs.end());
    std::vector<double> fr(fs.size(), 0.0);
    if (d.foff) fr = fs;
    if (e == hipSuccess) e = up(L.fr, fr.data(), fr.size() * 8);
    if (e == hipSuccess)
        e = c->precision == IBDVM_F32_STORE ? up(L.fsT, fs32.data(), fs32.size() * 4) : up(L.fsT, fs.data(), fs.size() * 8);
    std::vector<int> cflag32(g.cflag.begin(), g.cflag.end());
    {
        // second neighbours along x (and y in 3D), and the update records with
        // the flag word of the cell above along the marching axis (y in 2D, z
        // in 3D; the parameters are written on device)
        const int nx = c->prob.n[0], ny = c->prob.n[1], nz = D == 3 ? c->prob.n[2] : 1;
        const size_t nxy = (size_t)nx * ny;
        auto solid = [&](int i, int j, int k) {
            return i >= 0 && i < nx && j >= 0 && j < ny && (g.cflag[i + nx * j + nxy * k] & ibdvm::CF_SOLID);
        };
        std::vector<double> qrec((size_t)g.Nc * ibdvm::kQWords, 0.0);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    int &f = cflag32[i + nx * j + nxy * k];
                    if (solid(i - 2, j, k)) f |= ibdvm::CF_XM2;
                    if (solid(i + 2, j, k)) f |= ibdvm::CF_XP2;
                    if (D == 3 && solid(i, j - 2, k)) f |= ibdvm::CF_YM2;
                    if (D == 3 && solid(i, j + 2, k)) f |= ibdvm::CF_YP2;
                }
        const size_t up_stride = D == 2 ? (size_t)nx : nxy;
        const size_t up_word = D == 2 ? 8 : 9;
        for (size_t cc = 0; cc < (size_t)g.Nc; ++cc) {
            const int up_flags = cc + up_stride < (size_t)g.Nc ? cflag32[cc + up_stride] : 0;
            std::memcpy(&qrec[cc * ibdvm::kQWords + up_word], &up_flags, 4);
        }
        if (e == hipSuccess) e = up(L.cellq, qrec.data(), qrec.size() * 8);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e == hipSuccess) e = up(L.cflag, cflag32.data(), cflag32.size() * 4);
    if (e == hipSuccess) e = up(L.pnb, g.pnb.data(), g.pnb.size() * 4);
    if (e == hipSuccess) e = up(L.pairs, dp.data(), dp.size() * sizeof(ibdvm::DPair));
    if (e == hipSuccess) e = up(L.cls, g.cls.data(), g.cls.size());
    if (e == hipSuccess) e = up(L.wg, g.wg.data(), g.wg.size() * 8);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return fail(IBDVM_E_DEVICE, std::string("table upload: ") + hipGetErrorString(e));
    }
    st = reset_clock(c);
    if (!st) st = put_dev(c);
    const double *no_noise[2] = {nullptr, nullptr};
    if (!st) st = upload_state(c, nullptr, no_noise, 0.0);
    if (!st) st = refresh_moments(c);
    if (!st) st = sync_and_check(c);
    if (st) {
        delete c;
        return st;
    }
    *out = c;
    return IBDVM_OK;
}

void ibdvm_destroy(ibdvm_ctx *ctx) { delete ctx; }

ibdvm_status ibdvm_info(const ibdvm_ctx *c, int64_t out[7])
{
    if (!c || !out) return fail(IBDVM_E_INVALID_ARG, "null argument");
    out[0] = c->prob.dim;
    out[1] = c->geo.Nc;
    out[2] = c->geo.NV;
    out[3] = c->NA;
    out[4] = (int64_t)c->geo.pairs.size();
    out[5] = c->geo.nfluid;
    out[6] = c->geo.nghost;
    return IBDVM_OK;
}

ibdvm_status ibdvm_init_freestream(ibdvm_ctx *c, const double *u0, const double *u1, double amp)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = reset_clock(c))) return st;
    const double *noise[2] = {u0, c->NA == 2 ? u1 : nullptr};
    if ((st = upload_state(c, nullptr, noise, amp))) return st;
    if ((st = refresh_moments(c))) return st;
    return sync_and_check(c);
}

ibdvm_status ibdvm_init_freestream_hashed(ibdvm_ctx *c, uint64_t seed, double amp)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = reset_clock(c))) return st;
    for (int A = 0; A < c->NA; ++A)
        HIP_CHECK(ibdvm::launch_state_hashed(c->dev, c->precision, c->cur, A, (unsigned long long)seed, amp, c->stream));
    if ((st = refresh_moments(c))) return st;
    return sync_and_check(c);
}

ibdvm_status ibdvm_set_state(ibdvm_ctx *c, const double *f0, const double *f1)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    if (!f0 || (c->NA == 2 && !f1)) return fail(IBDVM_E_INVALID_ARG, "null state array");
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = reset_clock(c))) return st;
    const double *src[2] = {f0, f1};
    if ((st = upload_state(c, src, nullptr, 0.0))) return st;
    if ((st = refresh_moments(c))) return st;
    return sync_and_check(c);
}

ibdvm_status ibdvm_get_state(ibdvm_ctx *c, double *f0, double *f1)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    if (!f0 || (c->NA == 2 && !f1)) return fail(IBDVM_E_INVALID_ARG, "null state array");
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = finish_pending(c))) return st;
    // stage through the free state buffer
    const long long NV = c->geo.NV, Nc = c->geo.Nc;
    char *stage = c->ws + c->L.f[c->cur ^ 1][0];
    size_t stage_bytes = c->L.state_bytes * c->NA;
    long long chunk_cells = std::max<long long>(1, (long long)(stage_bytes / (NV * 8)));
    double *dst[2] = {f0, f1};
    for (int A = 0; A < c->NA; ++A)
        for (long long c0 = 0; c0 < Nc; c0 += chunk_cells) {
            long long nc = std::min(chunk_cells, Nc - c0);
            HIP_CHECK(ibdvm::launch_state_get(c->dev, c->precision, c->cur, A, (double *)stage, c0 * NV, nc * NV, c->stream));
            HIP_CHECK(hipMemcpyAsync(dst[A] + c0 * NV, stage, nc * NV * 8, hipMemcpyDeviceToHost, c->stream));
            HIP_CHECK(hipStreamSynchronize(c->stream));
        }
    return sync_and_check(c);
}

namespace {
bool tile_supported(int dim, const ibdvm::Tile &t);

// checkpoint record: this header, the control block, the cell records
// (moments, then update parameters) and the stored state arrays, each at
// an 8-byte aligned offset in that order
struct CkptHeader {
    char magic[8];
    uint64_t fingerprint;
    int64_t Nc, NV, npairs, step;
    int32_t dim, NA, precision, V, TX, LY;
    uint64_t ctrl_bytes, cellp_bytes, cellq_bytes, state_bytes;
};
constexpr char kCkptMagic[8] = {'I', 'B', 'D', 'V', 'M', 'C', 'K', '1'};

// FNV-1a over the values that define a solve: a record restores only into
// a context of the same problem, physics and storage precision (each value
// hashed by its own bytes, arrays whole: no padding enters)
void fnv(uint64_t &h, const void *p, size_t n)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
}

uint64_t fingerprint(const ibdvm_ctx *c)
{
    const ibdvm::Problem &p = c->prob;
    uint64_t h = 14695981039346656037ull;
#define IBDVM_FP(x) fnv(h, &(x), sizeof(x))
    IBDVM_FP(p.dim), IBDVM_FP(p.n), IBDVM_FP(p.lo), IBDVM_FP(p.hi), IBDVM_FP(p.outer), IBDVM_FP(p.lid_u);
    IBDVM_FP(p.vn), IBDVM_FP(p.vlo), IBDVM_FP(p.vhi), IBDVM_FP(p.rule), IBDVM_FP(p.vstretch), IBDVM_FP(p.vref_amp);
    IBDVM_FP(p.vref_width), IBDVM_FP(p.vref_centre), IBDVM_FP(p.vweights), IBDVM_FP(p.gkind), IBDVM_FP(p.gcen);
    IBDVM_FP(p.gsize), IBDVM_FP(p.aoa), IBDVM_FP(p.flags), IBDVM_FP(p.Uw), IBDVM_FP(p.Ow);
    IBDVM_FP(c->Kn), IBDVM_FP(c->Ma), IBDVM_FP(c->Pr), IBDVM_FP(c->gam), IBDVM_FP(c->alpha), IBDVM_FP(c->Tw);
    IBDVM_FP(c->cfl), IBDVM_FP(c->omega), IBDVM_FP(c->avhs), IBDVM_FP(c->precision), IBDVM_FP(c->NA);
#undef IBDVM_FP
    return h;
}

size_t align8(size_t x) { return (x + 7) & ~size_t(7); }

struct CkptSizes {
    size_t ctrl, cellp, cellq, state, total;
};

CkptSizes ckpt_sizes(const ibdvm_ctx *c)
{
    CkptSizes z;
    z.ctrl = sizeof(ibdvm::Ctrl);
    z.cellp = (size_t)c->geo.Nc * ibdvm::kCellWords * 8;
    z.cellq = (size_t)c->geo.Nc * ibdvm::kQWords * 8;
    z.state = c->L.state_bytes;
    z.total = align8(sizeof(CkptHeader)) + align8(z.ctrl) + align8(z.cellp) + align8(z.cellq) + (size_t)c->NA * align8(z.state);
    return z;
}
}  // namespace

ibdvm_status ibdvm_checkpoint_bytes(const ibdvm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(IBDVM_E_INVALID_ARG, "null argument");
    *bytes = ckpt_sizes(c).total;
    return IBDVM_OK;
}

ibdvm_status ibdvm_checkpoint(ibdvm_ctx *c, void *record, size_t bytes)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    if (!record) return fail(IBDVM_E_INVALID_ARG, "null record");
    const CkptSizes z = ckpt_sizes(c);
    if (bytes < z.total) return fail(IBDVM_E_INVALID_ARG, "checkpoint record smaller than ibdvm_checkpoint_bytes");
    HIP_CHECK(hipSetDevice(c->device));
    // the cell records of the current state are complete once its moment
    // finish has run; a non-physical state is not checkpointed
    if ((st = finish_pending(c)) || (st = sync_and_check(c))) return st;
    char *out = (char *)record;
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, sizeof(h.magic));
    h.fingerprint = fingerprint(c);
    h.Nc = c->geo.Nc, h.NV = c->geo.NV, h.npairs = (int64_t)c->geo.pairs.size(), h.step = c->step;
    h.dim = c->prob.dim, h.NA = c->NA, h.precision = c->precision;
    h.V = c->tile.V, h.TX = c->tile.TX, h.LY = c->tile.LY;
    h.ctrl_bytes = z.ctrl, h.cellp_bytes = z.cellp, h.cellq_bytes = z.cellq, h.state_bytes = z.state;
    std::memcpy(out, &h, sizeof(h));
    size_t off = align8(sizeof(CkptHeader));
    auto get = [&](size_t dev_off, size_t n) -> hipError_t {
        hipError_t e = hipMemcpyAsync(out + off, c->ws + dev_off, n, hipMemcpyDeviceToHost, c->stream);
        off += align8(n);
        return e;
    };
    HIP_CHECK(get(c->L.ctrl, z.ctrl));
    HIP_CHECK(get(c->L.cellp, z.cellp));
    HIP_CHECK(get(c->L.cellq, z.cellq));
    for (int A = 0; A < c->NA; ++A) HIP_CHECK(get(c->L.f[c->cur][A], z.state));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    return IBDVM_OK;
}

ibdvm_status ibdvm_restore(ibdvm_ctx *c, const void *record, size_t bytes)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    if (!record) return fail(IBDVM_E_INVALID_ARG, "null record");
    const CkptSizes z = ckpt_sizes(c);
    if (bytes < sizeof(CkptHeader)) return fail(IBDVM_E_INVALID_ARG, "checkpoint record too short");
    CkptHeader h;
    std::memcpy(&h, record, sizeof(h));
    if (std::memcmp(h.magic, kCkptMagic, sizeof(h.magic)) != 0) return fail(IBDVM_E_INVALID_ARG, "not a checkpoint record");
    if (h.fingerprint != fingerprint(c) || h.Nc != c->geo.Nc || h.NV != c->geo.NV ||
        h.npairs != (int64_t)c->geo.pairs.size() || h.dim != c->prob.dim || h.NA != c->NA || h.precision != c->precision ||
        h.ctrl_bytes != z.ctrl || h.cellp_bytes != z.cellp || h.cellq_bytes != z.cellq || h.state_bytes != z.state)
        return fail(IBDVM_E_INVALID_ARG, "checkpoint of a different problem, precision or size");
    if (bytes < z.total) return fail(IBDVM_E_INVALID_ARG, "checkpoint record truncated");
    const ibdvm::Tile t{h.V, h.TX, h.LY};
    if (!tile_supported(c->prob.dim, t) || h.step < 0) return fail(IBDVM_E_INVALID_ARG, "corrupt checkpoint header");
    HIP_CHECK(hipSetDevice(c->device));
    // nothing of the context's own may still be writing these buffers
    HIP_CHECK(hipStreamSynchronize(c->stream));
    const char *in = (const char *)record;
    size_t off = align8(sizeof(CkptHeader));
    auto put = [&](size_t dev_off, size_t n) -> hipError_t {
        hipError_t e = hipMemcpyAsync(c->ws + dev_off, in + off, n, hipMemcpyHostToDevice, c->stream);
        off += align8(n);
        return e;
    };
    HIP_CHECK(put(c->L.ctrl, z.ctrl));
    HIP_CHECK(put(c->L.cellp, z.cellp));
    HIP_CHECK(put(c->L.cellq, z.cellq));
    for (int A = 0; A < c->NA; ++A) HIP_CHECK(put(c->L.f[c->cur][A], z.state));
    c->step = h.step;
    c->pending = false;
    c->res_valid = false;
    c->fin_cells = own_fin_cells(c);
    c->tile = t;
    c->dev.nchunk = (c->geo.NV + 64 * t.V - 1) / (64 * t.V);
    if ((st = put_dev(c))) return st;
    return sync_and_check(c);
}

ibdvm_status ibdvm_step(ibdvm_ctx *c, int32_t nsteps)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    if (nsteps < 0) return fail(IBDVM_E_INVALID_ARG, "negative step count");
    HIP_CHECK(hipSetDevice(c->device));
    for (int32_t i = 0; i < nsteps; ++i)
        if ((st = one_step(c))) return st;
    return finish_pending(c);
}

struct ibdvm_graph {
    std::vector<ibdvm_ctx *> ctxs;
    std::vector<int> cur0, parity0;  // buffer and tau slot the captured launches address
    int32_t nsteps = 0;
    bool fused = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
// captures nsteps steps of the contexts (one context: its own launches; more:
// the fused launches) on their stream, starting and ending with the moments
// finished, as ibdvm_step and ibdvm_batch_step leave them
ibdvm_status capture(ibdvm_ctx *const *cs, int32_t n, int32_t nsteps, bool fused, ibdvm_graph **out)
{
    if (!out) return fail(IBDVM_E_INVALID_ARG, "null output");
    *out = nullptr;
    if (n < 1) return fail(IBDVM_E_INVALID_ARG, "empty batch");
    if (nsteps < 2 || (nsteps & 1)) return fail(IBDVM_E_INVALID_ARG, "graph step count must be even and >= 2");
    for (int32_t i = 0; i < n; ++i)
        if (cs[i]->profiling) return fail(IBDVM_E_STATE, "profiling is on; turn it off before capturing");
    hipStream_t stream = cs[0]->stream;
    if (!stream) return fail(IBDVM_E_STATE, "capture needs a stream other than the legacy default stream");
    HIP_CHECK(hipSetDevice(cs[0]->device));
    ibdvm_status st = IBDVM_OK;
    if (fused)
        st = fused_fill(cs, n, false, stream);
    else
        st = finish_pending(cs[0]);
    if (st) return st;
    HIP_CHECK(hipStreamSynchronize(stream));
    auto *g = new ibdvm_graph;
    g->nsteps = nsteps;
    g->fused = fused;
    std::vector<long long> step0(n);
    for (int32_t i = 0; i < n; ++i) {
        g->ctxs.push_back(cs[i]);
        g->cur0.push_back(cs[i]->cur);
        g->parity0.push_back((int)(cs[i]->step & 1));
        step0[i] = cs[i]->step;
    }
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int32_t k = 0; k < nsteps && !st; ++k) st = fused ? fused_step(cs, n, stream) : one_step(cs[0]);
        if (!st) st = fused ? fused_fill(cs, n, false, stream) : finish_pending(cs[0]);
        hipError_t e2 = hipStreamEndCapture(stream, &g->graph);
        if (!st && e2 != hipSuccess) e = e2;
    }
    // capturing records the launches without running them
    for (int32_t i = 0; i < n; ++i) {
        cs[i]->cur = g->cur0[i];
        cs[i]->step = step0[i];
        cs[i]->pending = false;
    }
    if (e == hipSuccess && !st) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess || st) {
        (void)hipGetLastError();  // leave no stale error for the next launch check
        ibdvm_graph_destroy(g);
        return st ? st : fail(IBDVM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *out = g;
    return IBDVM_OK;
}
}  // namespace

ibdvm_status ibdvm_graph_create(ibdvm_ctx *c, int32_t nsteps, ibdvm_graph **out)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    return capture(&c, 1, nsteps, false, out);
}

ibdvm_status ibdvm_batch_graph_create(ibdvm_ctx *const *ctxs, int32_t n, int32_t nsteps, ibdvm_graph **out)
{
    ibdvm_status st = check_batch(ctxs, n);
    if (st) return st;
    return capture(ctxs, n, nsteps, true, out);
}

ibdvm_status ibdvm_graph_launch(ibdvm_graph *g)
{
    if (!g || !g->exec) return fail(IBDVM_E_INVALID_ARG, "null graph");
    const int n = (int)g->ctxs.size();
    for (int i = 0; i < n; ++i) {
        ibdvm_ctx *c = g->ctxs[i];
        ibdvm_status st = require_device(c);
        if (st) return st;
        if (c->cur != g->cur0[i] || (int)(c->step & 1) != g->parity0[i])
            return fail(IBDVM_E_STATE, "context advanced by an odd number of steps since the capture");
    }
    HIP_CHECK(hipSetDevice(g->ctxs[0]->device));
    ibdvm_status st = g->fused ? fused_fill(g->ctxs.data(), n, false, g->ctxs[0]->stream) : finish_pending(g->ctxs[0]);
    if (st) return st;
    HIP_CHECK(hipGraphLaunch(g->exec, g->ctxs[0]->stream));
    for (ibdvm_ctx *c : g->ctxs) {
        c->step += g->nsteps;
        c->res_valid = true;
    }
    return IBDVM_OK;
}

void ibdvm_graph_destroy(ibdvm_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

ibdvm_status ibdvm_residual(ibdvm_ctx *c, double res[6])
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    if (!res) return fail(IBDVM_E_INVALID_ARG, "null output");
    if (!c->res_valid) return fail(IBDVM_E_STATE, "no step since the state was set");
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = finish_pending(c))) return st;
    constexpr int R = ibdvm::kResVars;
    const size_t nb = (size_t)((c->geo.Nc + c->fin_cells - 1) / c->fin_cells);
    std::vector<double> part(nb * 2 * R);
    HIP_CHECK(hipMemcpyAsync(part.data(), c->dev.respart, part.size() * 8, hipMemcpyDeviceToHost, c->stream));
    if ((st = sync_and_check(c))) return st;
    double num[R] = {0, 0, 0, 0, 0}, den[R] = {0, 0, 0, 0, 0};
    for (size_t b = 0; b < nb; ++b)
        for (int i = 0; i < R; ++i) {
            num[i] += part[b * 2 * R + i];
            den[i] += part[b * 2 * R + R + i];
        }
    double mx = 0.0;
    for (int i = 0; i < R; ++i) {
        // a momentum component that vanishes everywhere (U_z in 2D) has no residual
        res[i] = den[i] > 0.0 ? std::sqrt(num[i]) / den[i] : 0.0;
        mx = std::max(mx, res[i]);
    }
    res[R] = mx;
    return IBDVM_OK;
}

ibdvm_status ibdvm_set_stream(ibdvm_ctx *c, void *stream)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = finish_pending(c))) return st;
    HIP_CHECK(hipStreamSynchronize(c->stream));
    c->stream = (hipStream_t)stream;
    return IBDVM_OK;
}

ibdvm_status ibdvm_batch_step(ibdvm_ctx *const *ctxs, int32_t n, int32_t nsteps)
{
    ibdvm_status st = check_batch(ctxs, n);
    if (st) return st;
    if (nsteps < 0) return fail(IBDVM_E_INVALID_ARG, "negative step count");
    if (n == 0) return IBDVM_OK;
    HIP_CHECK(hipSetDevice(ctxs[0]->device));
    for (int32_t k = 0; k < nsteps; ++k)
        if ((st = fused_step(ctxs, n, ctxs[0]->stream))) return st;
    return fused_fill(ctxs, n, false, ctxs[0]->stream);
}

ibdvm_status ibdvm_moments(ibdvm_ctx *c, double *out, int32_t out_is_device)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    if (!out) return fail(IBDVM_E_INVALID_ARG, "null output");
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = finish_pending(c))) return st;
    if (out_is_device) {
        HIP_CHECK(ibdvm::launch_moments_out(c->dev, out, c->stream));
        return IBDVM_OK;
    }
    double *stage = c->dev.part;  // holds no pending data once moments are final
    HIP_CHECK(ibdvm::launch_moments_out(c->dev, stage, c->stream));
    HIP_CHECK(hipMemcpyAsync(out, stage, (size_t)c->geo.Nc * 8 * 8, hipMemcpyDeviceToHost, c->stream));
    return sync_and_check(c);
}

ibdvm_status ibdvm_clock(ibdvm_ctx *c, double *dt, double *time, int64_t *step)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = sync_and_check(c))) return st;
    ibdvm::Ctrl ctrl;
    HIP_CHECK(hipMemcpy(&ctrl, c->ws + c->L.ctrl, sizeof(ctrl), hipMemcpyDeviceToHost));
    if (dt) *dt = ctrl.dt;
    if (time) *time = ctrl.time;
    if (step) *step = ctrl.step;
    return IBDVM_OK;
}

ibdvm_status ibdvm_wall_state(ibdvm_ctx *c, double *ghost, double *face, double *rho_w)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = finish_pending(c))) return st;
    HIP_CHECK(ibdvm::launch_fill_fin(c->dev, c->precision, c->cur, (int)(c->step & 1), true, false, c->stream));
    const size_t np = c->geo.pairs.size(), n = np * c->geo.NV;
    if (np) {
        for (int A = 0; A < c->NA; ++A) {
            if (ghost) HIP_CHECK(hipMemcpyAsync(ghost + A * n, c->dev.ghost[A], n * 8, hipMemcpyDeviceToHost, c->stream));
            if (face) HIP_CHECK(hipMemcpyAsync(face + A * n, c->dev.face[A], n * 8, hipMemcpyDeviceToHost, c->stream));
        }
        if (rho_w) HIP_CHECK(hipMemcpyAsync(rho_w, c->dev.rhow, np * 8, hipMemcpyDeviceToHost, c->stream));
    }
    return sync_and_check(c);
}

ibdvm_status ibdvm_surface_forces(ibdvm_ctx *c, double force[3], double *C_D, double *C_L, ibdvm_wall_point *pts,
                                  int32_t cap, int32_t *n_pts)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = finish_pending(c))) return st;
    const size_t np = c->geo.pairs.size();
    HIP_CHECK(ibdvm::launch_fill_fin(c->dev, c->precision, c->cur, (int)(c->step & 1), true, false, c->stream));
    HIP_CHECK(ibdvm::launch_force(c->dev, c->precision, c->cur, c->stream));
    constexpr int KW = ibdvm::kForceWords;
    std::vector<double> pf(np * KW), rw(np);
    if (np) {
        HIP_CHECK(hipMemcpyAsync(pf.data(), c->dev.pforce, np * KW * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_CHECK(hipMemcpyAsync(rw.data(), c->dev.rhow, np * 8, hipMemcpyDeviceToHost, c->stream));
    }
    if ((st = sync_and_check(c))) return st;
    double F[3] = {0, 0, 0};
    for (size_t p = 0; p < np; ++p)
        for (int b = 0; b < 3; ++b) F[b] += pf[KW * p + b];
    if (force)
        for (int b = 0; b < 3; ++b) force[b] = F[b];
    double qd = 0.5 * c->Uinf * c->Uinf * c->Lref;
    if (C_D) *C_D = qd > 0 ? F[0] / qd : NAN;
    if (C_L) *C_L = qd > 0 ? F[1] / qd : NAN;
    int32_t m = 0;
    if (pts)
        for (size_t p = 0; p < np && m < cap; ++p, ++m) {
            const ibdvm::PairGeom &g = c->geo.pairs[p];
            for (int b = 0; b < 3; ++b) {
                pts[m].xw[b] = g.xw[b];
                pts[m].nw[b] = g.nw[b];
            }
            pts[m].rho_w = rw[p];
            pts[m].p_w = pf[KW * p + 3];
            for (int b = 0; b < 3; ++b) pts[m].tau_w[b] = pf[KW * p + 4 + b];
            pts[m].q_n = pf[KW * p + 7];
            // Section 4: C_p = 2 (p_w - p_0) / (rho_0 U_0^2), freestream p_0 = rho_0 T_0 / 2 = 1/2
            pts[m].C_p = c->Uinf > 0 ? 2.0 * (pts[m].p_w - 0.5) / (c->Uinf * c->Uinf) : NAN;
            // gas at the wall point: rho, U from the raw moments, then
            // T = 4 (rho E - rho |U|^2 / 2) / (3 rho) with rho E = sum w e / 2
            const double *r = &pf[KW * p + 8];
            double u2 = 0.0;
            for (int b = 0; b < 3; ++b) {
                pts[m].u_s[b] = b < c->prob.dim ? r[1 + b] / r[0] : 0.0;
                u2 += pts[m].u_s[b] * pts[m].u_s[b];
            }
            pts[m].T_s = 4.0 * (0.5 * r[4] - 0.5 * r[0] * u2) / (3.0 * r[0]);
        }
    if (n_pts) *n_pts = pts ? m : (int32_t)np;
    return IBDVM_OK;
}

ibdvm_status ibdvm_surface_forces_static(ibdvm_ctx *c, double *out, int32_t cap)
{
    if (!c) return fail(IBDVM_E_INVALID_ARG, "null context");
    if (!out || cap < 0) return fail(IBDVM_E_INVALID_ARG, "null output or negative capacity");
    const size_t np = c->geo.pairs.size();
    if (np > (size_t)ibdvm::kStaticMaxPairs)
        return fail(IBDVM_E_INVALID_ARG, "the solve has " + std::to_string(np) + " ghost-donor pairs, more than the " +
                                             std::to_string(ibdvm::kStaticMaxPairs) +
                                             " the static scratch of ibdvm_surface_forces_static holds");
    ibdvm_status st = require_device(c);
    if (st) return st;
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = finish_pending(c))) return st;
    HIP_CHECK(ibdvm::launch_fill_fin(c->dev, c->precision, c->cur, (int)(c->step & 1), true, false, c->stream));
    HIP_CHECK(ibdvm::launch_force_static(c->dev, c->precision, c->cur, out, cap, 0.5 * c->Uinf * c->Uinf * c->Lref,
                                         c->Uinf, c->stream));
    return IBDVM_OK;
}

namespace {
// TX grid columns per workgroup: 2D 4 or 8 (a row of columns); 3D 16 or 8
// (a 4 x 4 or 4 x 2 tile of columns)
bool tile_supported(int dim, const ibdvm::Tile &t)
{
    bool tx = dim == 2 ? (t.TX == 4 || t.TX == 8) : (t.TX == 16 || t.TX == 8);
    bool v = t.V == 1 || t.V == 2;
    return tx && v && t.LY >= 1 && t.LY <= 256;
}

hipError_t launch_update_tile(const ibdvm::Dev &d, int dim, int precision, int cur, int slot, const ibdvm::Tile &t,
                              hipStream_t s)
{
    return dim == 2 ? ibdvm::launch_update2d(d, precision, cur, slot, t, s)
                    : ibdvm::launch_update3d(d, precision, cur, slot, t, s);
}
}  // namespace

ibdvm_status ibdvm_set_tile(ibdvm_ctx *c, int32_t V, int32_t TX, int32_t LY)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    ibdvm::Tile t{V, TX, LY};
    if (!tile_supported(c->prob.dim, t)) return fail(IBDVM_E_INVALID_ARG, "unsupported tile");
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = finish_pending(c))) return st;
    c->tile = t;
    c->dev.nchunk = (c->geo.NV + 64 * V - 1) / (64 * V);
    return put_dev(c);
}

ibdvm_status ibdvm_get_tile(const ibdvm_ctx *c, int32_t out[3])
{
    if (!c || !out) return fail(IBDVM_E_INVALID_ARG, "null argument");
    out[0] = c->tile.V;
    out[1] = c->tile.TX;
    out[2] = c->tile.LY;
    return IBDVM_OK;
}

ibdvm_status ibdvm_autotune(ibdvm_ctx *c, int32_t reps, int32_t out[3])
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    if (reps < 1) return fail(IBDVM_E_INVALID_ARG, "reps must be positive");
    HIP_CHECK(hipSetDevice(c->device));
    if ((st = finish_pending(c))) return st;
    // the update kernel reads the current state and writes the other buffer
    // and the partial moments; neither is live here, so timing it leaves the
    // solve unchanged once the control block is restored
    ibdvm::Ctrl saved;
    HIP_CHECK(hipStreamSynchronize(c->stream));
    HIP_CHECK(hipMemcpy(&saved, c->ws + c->L.ctrl, sizeof(saved), hipMemcpyDeviceToHost));
    const int slot = (int)(c->step & 1);
    ibdvm::Tile best = c->tile;
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    const int dim = c->prob.dim;
    const int Vs[2] = {1, 2}, TXs[2] = {dim == 2 ? 4 : 16, 8};
    const int LYs[3] = {dim == 2 ? 32 : 16, dim == 2 ? 64 : 48, dim == 2 ? 120 : 256};
    for (int V : Vs)
        for (int TX : TXs)
            for (int LY : LYs) {
                ibdvm::Tile t{V, TX, LY};
                if (!tile_supported(dim, t)) continue;
                ibdvm::Dev d = c->dev;
                d.nchunk = (c->geo.NV + 64 * V - 1) / (64 * V);
                HIP_CHECK(launch_update_tile(d, dim, c->precision, c->cur, slot, t, c->stream));
                HIP_CHECK(hipEventRecord(e0, c->stream));
                for (int r = 0; r < reps; ++r) HIP_CHECK(launch_update_tile(d, dim, c->precision, c->cur, slot, t, c->stream));
                HIP_CHECK(hipEventRecord(e1, c->stream));
                HIP_CHECK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < 0.99f * best_ms) {  // ties within 1 % keep the earlier candidate, so repeated runs agree
                    best_ms = ms;
                    best = t;
                }
            }
    HIP_CHECK(hipEventDestroy(e0));
    HIP_CHECK(hipEventDestroy(e1));
    HIP_CHECK(hipMemcpy(c->ws + c->L.ctrl, &saved, sizeof(saved), hipMemcpyHostToDevice));
    c->tile = best;
    c->dev.nchunk = (c->geo.NV + 64 * best.V - 1) / (64 * best.V);
    if ((st = put_dev(c))) return st;
    if (out) {
        out[0] = best.V;
        out[1] = best.TX;
        out[2] = best.LY;
    }
    return IBDVM_OK;
}

ibdvm_status ibdvm_profile(ibdvm_ctx *c, int32_t enable)
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    HIP_CHECK(hipSetDevice(c->device));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    for (auto &v : c->ev) {
        for (hipEvent_t e : v) HIP_CHECK(hipEventDestroy(e));
        v.clear();
    }
    c->profiling = enable != 0;
    return IBDVM_OK;
}

ibdvm_status ibdvm_profile_read(ibdvm_ctx *c, double ms[2], int64_t counts[2])
{
    ibdvm_status st = require_device(c);
    if (st) return st;
    if (!ms || !counts) return fail(IBDVM_E_INVALID_ARG, "null output");
    HIP_CHECK(hipSetDevice(c->device));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    for (int kind = 0; kind < 2; ++kind) {
        std::vector<hipEvent_t> &v = c->ev[kind];
        double total = 0.0;
        for (size_t i = 0; i + 1 < v.size(); i += 2) {
            float t = 0.f;
            HIP_CHECK(hipEventElapsedTime(&t, v[i], v[i + 1]));
            total += t;
        }
        ms[kind] = total;
        counts[kind] = (int64_t)(v.size() / 2);
        for (hipEvent_t e : v) HIP_CHECK(hipEventDestroy(e));
        v.clear();
    }
    return IBDVM_OK;
}

ibdvm_status ibdvm_stream_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    if (!src || !dst) return fail(IBDVM_E_INVALID_ARG, "null buffer");
    if (bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
        return fail(IBDVM_E_INVALID_ARG, "copy size and addresses must be multiples of 16 bytes");
    HIP_CHECK(ibdvm::launch_stream_copy(src, dst, (long long)(bytes / 16), (hipStream_t)stream));
    return IBDVM_OK;
}

ibdvm_status ibdvm_index_sets(const ibdvm_ctx *c, uint8_t *solid, int32_t *pairs, uint8_t *cls)
{
    if (!c) return fail(IBDVM_E_INVALID_ARG, "null context");
    const ibdvm::Geometry &g = c->geo;
    if (solid)
        for (int i = 0; i < g.Nc; ++i) solid[i] = g.cflag[i] & ibdvm::CF_SOLID;
    for (size_t p = 0; p < g.pairs.size(); ++p) {
        const ibdvm::PairGeom &q = g.pairs[p];
        if (pairs) {
            int32_t *o = pairs + 32 * p;
            o[0] = q.gc;
            o[1] = q.dc;
            o[2] = q.ac;
            o[3] = q.axis;
            o[4] = q.sign;
            o[5] = q.ns;
            for (int j = 0; j < 26; ++j) o[6 + j] = j < q.ns ? q.sc[j] : -1;
        }
    }
    if (cls && !g.cls.empty()) std::memcpy(cls, g.cls.data(), g.cls.size());
    return IBDVM_OK;
}

ibdvm_status ibdvm_pair_geometry(const ibdvm_ctx *c, double *g9, double *wg)
{
    if (!c) return fail(IBDVM_E_INVALID_ARG, "null context");
    const ibdvm::Geometry &g = c->geo;
    for (size_t p = 0; p < g.pairs.size(); ++p) {
        if (!g9) break;
        for (int b = 0; b < 3; ++b) {
            g9[9 * p + b] = g.pairs[p].xw[b];
            g9[9 * p + 3 + b] = g.pairs[p].nw[b];
            g9[9 * p + 6 + b] = g.pairs[p].xsp[b];
        }
    }
    if (wg && !g.wg.empty()) std::memcpy(wg, g.wg.data(), g.wg.size() * 8);
    return IBDVM_OK;
}

}  // extern "C"
