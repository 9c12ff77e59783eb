/*
 * ibdvm.h -- C ABI of the MI355X immersed-boundary discrete-velocity step.
 *
 * The library advances the discrete velocity model of the Shakhov equation
 * (arXiv 2512.20252, Section 2.2 semi-discrete form with the forward Euler
 * march of Section 4) on a uniform Cartesian grid with a ghost-cell immersed
 * boundary (Section 3.2: upwind-weighted compact interpolation, Maxwell
 * gas-surface interaction of Section 2.3, velocity-space cut-cell correction
 * of Section 3.2.3).  2D problems use the reduced distributions h, b of
 * Section 4; 3D problems carry the full distribution f.
 *
 * Units follow Section 4: lengths in the coordinate unit (Kn is relative to
 * it), velocities in sqrt(2 R T_inf), rho_inf = T_inf = 1, p = rho T / 2,
 * freestream velocity (Ma sqrt(gamma/2), 0, 0).
 *
 * Memory and ownership
 *   - All device memory is the caller's: one device buffer of at least
 *     ibdvm_footprint() bytes passed in ibdvm_opts.workspace.  The library
 *     never allocates device memory; ibdvm_destroy frees only the host-side
 *     context.
 *   - The caller owns the HIP stream (ibdvm_opts.stream, a hipStream_t; NULL
 *     is the null stream).  ibdvm_step only enqueues work on it.
 *   - Host arrays passed in are read before the call returns; host arrays
 *     passed out are written before the call returns.
 *   - Array layouts: cell c = i + n0*(j + n1*l) (x fastest); velocity node
 *     k = ix + N0*(iy + N1*iz); distributions [cell][node], node innermost.
 *
 * Errors
 *   - Every entry point returns an ibdvm_status; no exception crosses the ABI.
 *     ibdvm_last_error() returns a thread-local message for the last failure.
 *   - A context whose device health word reports NaN, rho <= 0 or T <= 0
 *     returns IBDVM_E_UNSTABLE at the next synchronising call and then
 *     IBDVM_E_STATE for every compute call until it is destroyed.
 *   - One context is used by one host thread at a time; distinct contexts
 *     are independent.
 */
#ifndef IBDVM_H
#define IBDVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibdvm_ctx ibdvm_ctx;

typedef enum {
    IBDVM_OK = 0,
    IBDVM_E_INVALID_ARG = 1, /* a parameter is out of range or a pointer is NULL */
    IBDVM_E_GEOMETRY = 2,    /* body too close to the outer boundary (< 3 cells) */
    IBDVM_E_NO_MEMORY = 3,   /* workspace smaller than ibdvm_footprint() */
    IBDVM_E_DEVICE = 4,      /* a HIP runtime call failed */
    IBDVM_E_UNSTABLE = 5,    /* the device health word reported NaN, rho<=0 or T<=0 */
    IBDVM_E_UNSUPPORTED = 6, /* combination not implemented */
    IBDVM_E_STATE = 7,       /* context unusable (host-only or previously unstable) */
    IBDVM_E_CANCELLED = 8    /* serving: the request was cancelled (ibdvm_server_cancel) */
} ibdvm_status;

/* outer boundary of the box: freestream ghost cells (Section 4 external
 * flows), periodic, or (2D only) diffuse walls at T_w on all four sides with
 * the wall y = hi moving along +x at lid_u (lid-driven cavity, Section 4):
 * the wall model of Section 2.3 applied at the domain faces, with the wall
 * density from zero normal mass flux through each boundary face; or (2D
 * only) specular walls on all four sides (the Section 2.3 model with
 * alpha = 0): a boundary cell's velocities leaving the wall see its own
 * value at the mirrored velocity, so the walls pass no mass and no energy
 * (needs a velocity grid symmetric about 0, which every grid here is) */
enum { IBDVM_OUTER_FREESTREAM = 0, IBDVM_OUTER_PERIODIC = 1, IBDVM_OUTER_WALLS = 2, IBDVM_OUTER_SPECULAR = 3 };
enum { IBDVM_RULE_MIDPOINT = 0, IBDVM_RULE_TRAPEZOID = 1, IBDVM_RULE_STRETCHED = 2, IBDVM_RULE_REFINED = 3 };
/* node weights of the mapped grids (ibdvm_vgrid.weights) */
enum { IBDVM_WEIGHTS_CELL = 0, IBDVM_WEIGHTS_JACOBIAN = 1 };
enum {
    IBDVM_GEOM_NONE = 0,
    IBDVM_GEOM_CIRCLE = 1,  /* 2D, size[0] = radius */
    IBDVM_GEOM_ELLIPSE = 2, /* 2D, size[0], size[1] = semi-axes, rotated by aoa about the centre */
    IBDVM_GEOM_AIRFOIL = 3, /* 2D, centre = leading edge, size[0] = chord, size[1] = thickness ratio */
    IBDVM_GEOM_SPHERE = 4   /* 3D, size[0] = radius */
};
enum { IBDVM_F64 = 0, IBDVM_F32_STORE = 1 };
enum {
    IBDVM_FLAG_NO_CUTCELL = 1u << 0, /* ablation: classify velocity cells by node sign only */
    IBDVM_FLAG_NO_UPWIND = 1u << 1,  /* ablation: uniform weights 1/N_S in the ghost interpolation */
    /* semi-implicit collision for small Kn (a variant; the paper marches
     * with forward Euler, Section 4): each step transports explicitly, then
     * relaxes implicitly, f = (f* + r g^S)/(1 + r) with r = dt/tau, where
     * rho, U, T and tau come from the transported state f* and the heat flux
     * of g^S is q* / (1 + Pr r) (the Shakhov equilibrium carries (1 - Pr) q,
     * Section 2.1); dt = cfl / sum_a max|xi_a|/dx_a, without the
     * relaxation-time bound */
    IBDVM_FLAG_IMPLICIT_COLLISION = 1u << 2,
    /* positivity option of the ghost-side face value: taken on the
     * shifted-point -> wall line of Section 3.2.1 no further than the wall
     * when the face lies beyond it (inside the solid); without it the face
     * value is that line's value at the face (second order on smooth data) */
    IBDVM_FLAG_FACE_LIMIT = 1u << 3,
    /* ablation of Section 3.3.3: the intermediate ghost value is the naive
     * linear extrapolation of donor and auxiliary cell along the pair's axis,
     * f_gc = 2 f_dc - f_ac, instead of the upwind-weighted surface-cell
     * interpolation of Section 3.2.2 */
    IBDVM_FLAG_NAIVE_EXTRAPOLATION = 1u << 4,
    /* ablation: no donor slope, the shifted-point value of Section 3.2.1 is
     * the donor value (the construction used where no fluid auxiliary cell
     * exists, applied to every pair) */
    IBDVM_FLAG_NO_AUX_SLOPE = 1u << 5,
    /* 2D FP32 storage of f itself instead of its offset from the freestream
     * Maxwellian (the default, whose rounding scales with the departure
     * from the freestream): for flows with near-vacuum regions, such as
     * hypersonic wakes, where f is far below the freestream value at the
     * freestream's velocities and the offset would cancel its digits */
    IBDVM_FLAG_F32_ABSOLUTE = 1u << 6,
    IBDVM_FLAG_HOST_ONLY = 1u << 8   /* build the geometry tables only; no device work */
};

/* uniform cell-centred Cartesian grid; dim 2 or 3, n[a] >= 4 */
typedef struct {
    int32_t dim;
    int32_t n[3];
    double lo[3], hi[3];
    int32_t outer_bc;
    double lid_u; /* IBDVM_OUTER_WALLS: speed of the wall y = hi along +x (units of sqrt(2 R T_inf)); else ignored */
} ibdvm_grid;

/* tensor velocity grid (Section 2.2 quadrature): midpoint nodes at
 * lo + (i + 1/2) h with h = (hi - lo)/N, or trapezoid nodes lo + i h with
 * h = (hi - lo)/(N - 1) and half weights at the ends, or stretched nodes
 * (a tensor form of the locally refined velocity mesh of Section 4): the
 * midpoint grid of u in [-1, 1] mapped by x(u) = hi sinh(stretch u) /
 * sinh(stretch), finer near 0, each node's dual cell the image of its
 * u-cell and its weight that cell's width; 2 to 256 nodes per axis; the box
 * must be symmetric about 0 */
typedef struct {
    int32_t n[3];
    double lo[3], hi[3];
    int32_t rule;
    double stretch; /* IBDVM_RULE_STRETCHED: beta in (0, 20]; else ignored */
    /* IBDVM_RULE_REFINED (a locally refined tensor grid, the refined
     * velocity mesh of the Section 4 sphere case in tensor form): per axis a
     * node density 1 + refine_amp (exp(-(x/w)^2) + exp(-((x - c)/w)^2)),
     * w = refine_width, c = refine_centre[a] (one bump when c = 0; e.g. c =
     * U_inf on x refines around both the wall and the freestream
     * Maxwellians); nodes and dual cells are the images of the uniform
     * midpoint cells of u in [-1, 1] under the inverse of the normalised
     * cumulative density, each weight its cell's width; refine_amp >= 0,
     * refine_width > 0, |c| < hi; else ignored */
    double refine_amp, refine_width, refine_centre[3];
    /* node weights of IBDVM_RULE_STRETCHED and IBDVM_RULE_REFINED:
     * IBDVM_WEIGHTS_CELL, the width (area, volume) of the node's dual cell,
     * or IBDVM_WEIGHTS_JACOBIAN, the derivative of the map at the node
     * times the u-cell width 2/N per axis (the midpoint rule of the
     * integral in u, whose moments of smooth distributions are far more
     * accurate than those of the dual cells: on a refined grid with 32
     * nodes per axis the discrete Maxwellian's density error falls from
     * 6e-3 to 1e-6, so the relaxation conserves mass that closely); cut
     * cells keep their incident fraction of the dual cell.  Must be
     * IBDVM_WEIGHTS_CELL for the uniform rules.  For the mapped rules
     * IBDVM_WEIGHTS_JACOBIAN is the better choice wherever it was
     * measured (refined grids on a Ma-5 cylinder and a Ma-3.8 sphere,
     * a stretched grid on a Ma-0.5 cylinder); the dual-cell default keeps
     * the first reading of those rules. */
    int32_t weights;
} ibdvm_vgrid;

typedef struct {
    int32_t kind;
    double center[3];
    double size[3];
    double aoa_rad;
} ibdvm_geometry;

typedef struct {
    int32_t precision;      /* IBDVM_F64 or IBDVM_F32_STORE */
    double cfl;             /* time-step safety factor in (0, 1] */
    double omega_vhs;       /* viscosity exponent (0.81 for argon, Section 4) */
    double a_vhs;           /* VSS/VHS alpha in the reference viscosity (1.0) */
    uint32_t flags;         /* IBDVM_FLAG_* */
    void *workspace;        /* device buffer, >= ibdvm_footprint() bytes, 256-byte aligned */
    size_t workspace_bytes;
    void *stream;           /* hipStream_t */
    /* velocity of the body's wall (Section 2.3 wall Maxwellian at (U_w,
     * T_w)) at wall point x_w: U_w + Omega_w x (x_w - centre), a translation
     * plus a rigid rotation about the geometry centre (2D: only Omega_w[2]
     * acts).  The velocity cells are still split by xi . n = 0 (Section
     * 3.2.3); zero for a wall at rest. */
    double U_w[3];
    double Omega_w[3];
} ibdvm_opts;

/* one wall point per ghost-donor pair: intersect point, unit normal n (into
 * the gas), wall density rho_w (Section 3.2.3), and moments of the wall
 * distribution f*_w in the frame of the grid (xi_n = xi . n): pressure p_w = sum w
 * xi_n^2 f*_w, shear stress tau_w = sum w xi_n (xi - xi_n n) f*_w (the
 * tangential part of the momentum flux), normal heat flux q_n = 1/2 sum w
 * xi_n (|xi|^2 h + b) (2D; 3D: |xi|^2 f), and the pressure coefficient of
 * Section 4, C_p = 2 (p_w - p_0) / (rho_0 U_0^2) with the freestream p_0 =
 * rho_0 T_0 / 2 = 1/2 (NaN when U_0 = 0); the temperature T_s and velocity
 * u_s of the gas at the wall point, the moments of f*_w (Section 2.1
 * definitions: the surface temperature and slip velocity Section 4 plots) */
typedef struct {
    double xw[3];
    double nw[3];
    double rho_w;
    double p_w;
    double tau_w[3];
    double q_n;
    double C_p;
    double T_s;
    double u_s[3];
} ibdvm_wall_point;

/* Bytes of device workspace a problem needs (state double buffer, per-cell
 * moments, geometry tables, per-pair buffers).  Host only; builds the
 * geometry to count pairs. */
ibdvm_status ibdvm_footprint(const ibdvm_grid *grid, const ibdvm_vgrid *vgrid, const ibdvm_geometry *geom,
                             const ibdvm_opts *opts, size_t *bytes);

/* Build a solve (Sections 3.2.1-3.2.3 for the geometry, Section 4 for the
 * constants): validates Kn > 0, Ma >= 0, Pr > 0, gamma > 1, 0 <= alpha <= 1,
 * T_w > 0; classifies cells, builds ghost-donor pairs, surface-cell lists
 * and cut-cell sets, uploads the tables into the workspace on the stream and
 * sets the state to the freestream Maxwellian.  With IBDVM_FLAG_HOST_ONLY
 * only the host tables are built (workspace may be NULL). */
ibdvm_status ibdvm_create(const ibdvm_grid *grid, const ibdvm_vgrid *vgrid, const ibdvm_geometry *geom, double Kn,
                          double Ma, double Pr, double gamma, double alpha, double T_w, const ibdvm_opts *opts,
                          ibdvm_ctx **out);

/* Frees the host context (not the workspace). */
void ibdvm_destroy(ibdvm_ctx *ctx);

/* Sizes: out[0..6] = dim, cells, velocity nodes, arrays per cell (2: h,b;
 * 1: f), pairs, fluid cells, ghost cells. */
ibdvm_status ibdvm_info(const ibdvm_ctx *ctx, int64_t out[7]);

/* State := freestream Maxwellian times (1 + amp * u), u given per (cell,
 * node) for each array (host, [cells][nodes] doubles); NULL arrays mean no
 * perturbation.  Synchronises. */
ibdvm_status ibdvm_init_freestream(ibdvm_ctx *ctx, const double *u0, const double *u1, double amp);

/* State := caller arrays (host doubles, [cells][nodes]; f1 ignored in 3D);
 * rounded to the storage precision.  Synchronises. */
ibdvm_status ibdvm_set_state(ibdvm_ctx *ctx, const double *f0, const double *f1);

/* Copies the state to host doubles.  Synchronises. */
ibdvm_status ibdvm_get_state(ibdvm_ctx *ctx, double *f0, double *f1);

/* Checkpoint and resume of the time march (Section 2.2) between steps.
 * ibdvm_set_state starts a new march from a state: it restarts the clock
 * and recomputes the moments with a summation order of its own.  A
 * checkpoint record instead holds everything the next step reads: the
 * stored state in its storage precision, the per-cell moment and
 * equilibrium records of that state, the clock (time, step, time-step
 * bookkeeping) and the update tile (the node-chunk width fixes the order of
 * the moment sums).  So a context restored from it takes the same steps as
 * the checkpointed one would have, bit for bit.
 *   ibdvm_checkpoint_bytes: the size of a record of this context (also on
 *     host-only contexts); state arrays dominate it.
 *   ibdvm_checkpoint: writes the record to caller host memory of at least
 *     that size (bytes); completes the pending moment finish; a context
 *     whose health word reports a non-physical state is refused with
 *     IBDVM_E_UNSTABLE and no record is written.
 *   ibdvm_restore: loads a record into a context created with the same
 *     grid, velocity grid, geometry, physics, options and precision (the
 *     record carries a fingerprint of them and the sizes; a mismatch, a
 *     truncated or foreign record gives IBDVM_E_INVALID_ARG and leaves the
 *     context as it was), and takes the record's tile.  Graphs captured on
 *     the context before the restore are refused afterwards if the step
 *     parity changed (IBDVM_E_STATE), as after any odd number of steps.
 * Both synchronise the context stream; the caller owns the record. */
ibdvm_status ibdvm_checkpoint_bytes(const ibdvm_ctx *ctx, size_t *bytes);
ibdvm_status ibdvm_checkpoint(ibdvm_ctx *ctx, void *record, size_t bytes);
ibdvm_status ibdvm_restore(ibdvm_ctx *ctx, const void *record, size_t bytes);

/* Enqueues nsteps forward-Euler steps on the context stream: ghost-cell
 * construction (Section 3.2), upwind MUSCL fluxes (Section 2.2) and Shakhov
 * relaxation with moments of the new state, time step
 * cfl / (sum_a max|xi_a|/dx_a + 1/tau_min). */
ibdvm_status ibdvm_step(ibdvm_ctx *ctx, int32_t nsteps);

/* Per-cell moments of the current state (Section 2.1): out[cell][8] =
 * rho, U0, U1, U2, T, q0, q1, q2 (NaN in solid cells).  out_is_device != 0:
 * out is a device pointer and the copy is enqueued on the stream; otherwise
 * host memory, and the call synchronises. */
ibdvm_status ibdvm_moments(ibdvm_ctx *ctx, double *out, int32_t out_is_device);

/* Force on the body from the momentum flux through the immersed-boundary
 * faces, drag and lift coefficients (reference length 2R for circle and
 * ellipse (major axis), chord for the airfoil, pi R^2 for the sphere) and up
 * to cap wall points.  Runs the ghost construction on the current state.
 * Synchronises. */
ibdvm_status ibdvm_surface_forces(ibdvm_ctx *ctx, double force[3], double *C_D, double *C_L, ibdvm_wall_point *pts,
                                  int32_t cap, int32_t *n_pts);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the outputs of ibdvm_surface_forces, computed the same way,
 * enqueued on the context stream and written to the device array out:
 * out[0..2] force, out[3] C_D, out[4] C_L, then for the first min(pairs,
 * cap) ghost-donor pairs 17 doubles each, the fields of ibdvm_wall_point in
 * order (x_w[3], n_w[3], rho_w, p_w, tau_w[3], q_n, C_p, T_s, u_s[3]); out
 * holds 5 + 17 cap doubles.  Allocates nothing and does not synchronise:
 * the per-pair force records live in a static device array of the library
 * that holds 16384 pairs (1.7 MB per device, kept until the process ends);
 * a solve with more pairs is refused with IBDVM_E_INVALID_ARG.  Calls on one
 * device share that array, so calls that overlap on one device (contexts on
 * different streams) race; calls ordered on one stream do not.  The device
 * health word is checked at the next synchronising call. */
ibdvm_status ibdvm_surface_forces_static(ibdvm_ctx *ctx, double *out, int32_t cap);

/* Time step of the last step, simulated time and step count.  Synchronises. */
ibdvm_status ibdvm_clock(ibdvm_ctx *ctx, double *dt, double *time, int64_t *step);

/* Geometry index sets (host copies; valid on host-only contexts):
 * solid[cells] (1 = centre inside the body); pairs[npairs][32] =
 * ghost, donor, auxiliary (-1: none), axis, sign, N_S, 26 surface cells
 * (-1 padded); cls[npairs][nodes] = 0 incident, 1 reflected, 2 cut with node
 * on the incident side, 3 cut with node on the reflected side.  Any output
 * pointer may be NULL. */
ibdvm_status ibdvm_index_sets(const ibdvm_ctx *ctx, uint8_t *solid, int32_t *pairs, uint8_t *cls);

/* Geometry FP64 tables (host copies): g9[npairs][9] = x_w, n_w, x_sp;
 * wg[npairs][nodes] = incident-side measure of each velocity dual cell. */
ibdvm_status ibdvm_pair_geometry(const ibdvm_ctx *ctx, double *g9, double *wg);

/* Runs the ghost construction on the current state and copies per-pair
 * buffers to host: ghost values and ghost-side face values
 * [arrays][npairs][nodes] and rho_w[npairs].  Synchronises. */
ibdvm_status ibdvm_wall_state(ibdvm_ctx *ctx, double *ghost, double *face, double *rho_w);

/* Convergence residual of the last step (Section 4): for each conservative
 * variable W_i = rho, rho U_x, rho U_y, rho U_z, rho E (rho E = rho |U|^2 / 2
 * + 3 rho T / 4), res[i] = sqrt(sum_cells (W_i^{n+1} - W_i^n)^2) /
 * sum_cells |W_i^{n+1}| over the fluid cells (0 for a component that is zero
 * everywhere), and res[5] = max_i res[i].  Sums in a fixed order.
 * IBDVM_E_STATE before the first step after the state was set.
 * Synchronises. */
ibdvm_status ibdvm_residual(ibdvm_ctx *ctx, double res[6]);

/* Rebinds the context to another stream of the same device (NULL: the
 * legacy default stream) after the work queued on its current stream has
 * finished (synchronises that stream).  Graphs captured earlier replay on
 * the new stream.  Serving uses it to move a solve prepared on its own
 * stream into a batch. */
ibdvm_status ibdvm_set_stream(ibdvm_ctx *ctx, void *stream);

/* Advances n contexts that share one stream and device by nsteps each
 * (serving form).  Each step is fused across the contexts: every ghost-fill
 * phase is one launch per (dimension, storage) group and the 2D update one
 * launch per (storage, V, TX) tile group, over the workgroups of all the
 * group's solves (at most 16 solves per launch); the 3D update is launched
 * per context.  Every solve does the same arithmetic as alone, so results
 * equal those of advancing each context alone bit for bit.  IBDVM_E_INVALID_ARG
 * if the contexts do not share a stream or one appears twice.  Only
 * enqueues; kernel timing (ibdvm_profile) is not recorded for these
 * launches. */
ibdvm_status ibdvm_batch_step(ibdvm_ctx *const *ctxs, int32_t n, int32_t nsteps);

/* Tile of the marching update kernel: V velocity nodes per lane (1 or 2),
 * TX grid columns per workgroup and LY rows (2D) or planes (3D) marched per
 * workgroup (1..256).  2D: TX = 4 or 8 adjacent columns.  3D: TX = 16 (a
 * 4 x 4 tile of columns) or 8 (4 x 2).  Unsupported values return
 * IBDVM_E_INVALID_ARG.  The tile fixes the order of the velocity sums, so
 * results are bit-identical only between runs with the same tile. */
ibdvm_status ibdvm_set_tile(ibdvm_ctx *ctx, int32_t V, int32_t TX, int32_t LY);
ibdvm_status ibdvm_get_tile(const ibdvm_ctx *ctx, int32_t out[3]);

/* Autotuner: times reps launches of the update kernel for every supported
 * tile on the current state (without advancing it), keeps the fastest and
 * returns it in out (may be NULL).  Synchronises. */
ibdvm_status ibdvm_autotune(ibdvm_ctx *ctx, int32_t reps, int32_t out[3]);

/* Kernel timing with HIP events (tracing aid).  While enabled, every
 * update launch and every ghost-fill / moment-finish launch of this context
 * is bracketed by a pair of events on the context stream.
 * ibdvm_profile_read synchronises, returns the summed durations in
 * milliseconds (ms[0] update kernel, ms[1] the ghost-fill phase: the
 * immersed-boundary fill with the moment finish and, with outer walls, the
 * wall ghost rows) and launch counts, and clears the record.  Disabling also
 * clears it. */
ibdvm_status ibdvm_profile(ibdvm_ctx *ctx, int32_t enable);
ibdvm_status ibdvm_profile_read(ibdvm_ctx *ctx, double ms[2], int64_t counts[2]);

/* Measurement: enqueues a plain streaming copy of `bytes` bytes from src to
 * dst (device pointers, 16-byte aligned, size a multiple of 16, buffers not
 * overlapping) on stream: every byte read once and written once with
 * coalesced 16-byte accesses.  Its rate is the practical HBM ceiling the
 * update kernels are compared with.  Only enqueues. */
ibdvm_status ibdvm_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Thread-local message describing the last failure on this thread. */
const char *ibdvm_last_error(void);

/* State := freestream Maxwellian times (1 + amp * u) with u uniform on
 * (-1, 1) from a counter-based generator on the device: the SplitMix64
 * output function of seed + (i + 1) * 0x9e3779b97f4a7c15, i running over
 * (array, cell, node) in storage order.  For inputs that need no host
 * arrays (serving).  Synchronises. */
ibdvm_status ibdvm_init_freestream_hashed(ibdvm_ctx *ctx, uint64_t seed, double amp);

/* ---------------------------------------------------------------- serving
 * Captured steps: nsteps (even, >= 2) steps of ctx recorded once as a HIP
 * graph and replayed on the context stream; a replay gives the same bits as
 * ibdvm_step(ctx, nsteps).  The graph addresses the context's buffers, so
 * it replays only while the context has advanced by an even number of steps
 * since the capture (IBDVM_E_STATE otherwise).  The context's stream must
 * not be the legacy default stream (IBDVM_E_STATE).  Launch only enqueues.
 * The graph must be destroyed before its context. */
typedef struct ibdvm_graph ibdvm_graph;
ibdvm_status ibdvm_graph_create(ibdvm_ctx *ctx, int32_t nsteps, ibdvm_graph **out);
/* The same for the fused steps of ibdvm_batch_step over n contexts sharing
 * a stream: one graph of nsteps fused steps; a replay advances every
 * context by nsteps and gives the bits of ibdvm_batch_step(ctxs, n, nsteps).
 * The graph must be destroyed before any of its contexts. */
ibdvm_status ibdvm_batch_graph_create(ibdvm_ctx *const *ctxs, int32_t n, int32_t nsteps, ibdvm_graph **out);
ibdvm_status ibdvm_graph_launch(ibdvm_graph *graph);
void ibdvm_graph_destroy(ibdvm_graph *graph);

/* Continuous batching of many 2D solves on one device (serving form).  The
 * server owns no device memory: it sub-allocates each admitted request's
 * footprint from the caller's workspace (256-byte aligned, kept by the
 * caller until ibdvm_server_destroy).  Requests are admitted in submission
 * order as soon as a block of their footprint and one of max_active slots
 * are free.  Solves below the fusion limit (ibdvm_server_set_fusion) form
 * the fused group on the server's stream: one captured graph of
 * steps_per_replay (K, even) fused steps over the group
 * (ibdvm_batch_graph_create) is replayed, and captured again whenever a
 * member joins or leaves.  Larger solves run standalone, each with its own
 * stream and captured graph of K steps, concurrently with the group.  A new
 * solve is created on its own stream while replays run and joins the group
 * at its next replay.  After each replay the C_D of every solve in it is
 * checked; a solve finishes when |C_D(n) - C_D(n - K)| < tol |C_D(n)|
 * (tol <= 0: never) or max_steps steps are done, and its memory and slot go back to the
 * queue.  A tile shape per (grid, velocity grid, precision)
 * is chosen once by ibdvm_autotune and reused.  Single-threaded: one thread
 * submits and polls. */
typedef struct ibdvm_server ibdvm_server;
typedef struct {
    int64_t id;
    int32_t status;    /* IBDVM_OK, or the error that ended the solve */
    int32_t converged; /* 1: C_D settled; 0: stopped at max_steps or failed */
    int64_t steps;
    double C_D, C_L;
    double t_submit, t_admit, t_done; /* seconds on the server clock */
    int64_t updates;                  /* fluid cells x velocity nodes x steps */
    int32_t tile[3];                  /* update tile used */
} ibdvm_result;

ibdvm_status ibdvm_server_create(void *workspace, size_t bytes, int32_t max_active, int32_t steps_per_replay,
                                 ibdvm_server **out);
/* Queues a solve (the problem arguments are those of ibdvm_create; opts'
 * workspace and stream are ignored).  The initial state is the freestream
 * times (1 + amp u) of ibdvm_init_freestream_hashed(seed).  moments_out
 * (host, [cells][8], may be NULL) receives the final moments and must stay
 * valid until the request is returned by poll.  IBDVM_E_NO_MEMORY if the
 * footprint exceeds the whole workspace. */
ibdvm_status ibdvm_server_submit(ibdvm_server *srv, const ibdvm_grid *grid, const ibdvm_vgrid *vgrid,
                                 const ibdvm_geometry *geom, double Kn, double Ma, double Pr, double gamma,
                                 double alpha, double T_w, const ibdvm_opts *opts, uint64_t seed, double amp,
                                 double tol, int64_t max_steps, double *moments_out, int64_t *id);
/* Advances the server: harvests finished replays, checks convergence,
 * admits queued requests, relaunches.  block != 0 waits until at least one
 * solve finishes (or none is active).  Returns up to cap finished results. */
ibdvm_status ibdvm_server_poll(ibdvm_server *srv, int32_t block, ibdvm_result *done, int32_t cap, int32_t *n_done);
/* Cancels request id, queued or active.  A queued request leaves the queue;
 * an active one waits for its replay in flight to end and is released: its
 * workspace block and slot go back to the queue at the next poll.  Either way
 * poll returns its result with status IBDVM_E_CANCELLED and the steps done
 * (moments_out is not written).  IBDVM_E_INVALID_ARG if no queued or active
 * request has this id (for instance one already finished).  Creating a
 * server, queueing and cancelling queued requests touch no device. */
ibdvm_status ibdvm_server_cancel(ibdvm_server *srv, int64_t id);
/* out = queued, active, finished, workspace bytes in use, workspace bytes. */
ibdvm_status ibdvm_server_info(const ibdvm_server *srv, int64_t out[5]);
double ibdvm_server_clock(const ibdvm_server *srv);
/* Solves with fewer than updates_per_step cell x node updates per step join
 * the fused group; larger ones run standalone (default 2^24; 0: none fused).
 * Applies to solves admitted afterwards. */
ibdvm_status ibdvm_server_set_fusion(ibdvm_server *srv, int64_t updates_per_step);
const char *ibdvm_server_error(const ibdvm_server *srv);
/* Waits for the active solves and releases them; queued ones are dropped. */
void ibdvm_server_destroy(ibdvm_server *srv);

#ifdef __cplusplus
}
#endif
#endif
