"""Throughput of the immersed-boundary Shakhov-DVM step on one MI355X.

One step = ghost construction for every ghost-donor pair, upwind MUSCL
fluxes, Shakhov relaxation and forward Euler update of every fluid cell and
velocity node, and the moments of the new state.  The workload is the 2D
cylinder at full size: [-8,8]^2 on 256x256 cells, radius 0.5, 48x48 midpoint
velocity grid on [-6,6]^2, Kn 0.1, Ma 0.3, freestream Maxwellian with seeded
1e-3 perturbation (synthetic input of the shape of the paper's cylinder
cases).

Prints one JSON line: cell-velocity updates/s of the FP64 step (the timed
steps replayed from a captured HIP graph, inputs resident in HBM), the
roofline of the update kernel (algorithmic HBM bytes per launch over its
HIP-event duration in eager steps of the same run), the FP32-storage form's rate and C_D difference, the
3D sphere at 96^3 x 24^3 in both forms, the lid-driven cavity at 256^2 x
100^2 in both forms, the semi-implicit collision against the explicit step on
the cylinder at Kn 2e-4, the FP32-storage and FP64 forms against the
oracle's converged C_D, the continuous-batching serving leg (the 128-request
stream of mixed solves), and the CPU oracle timed on this host over one step
of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
B_ALG = {(2, "f64"): 32, (2, "f32"): 16, (3, "f64"): 16, (3, "f32"): 8}


def _kernel_sha():
    with open(os.path.join(ROOT, "paper_2512_20252_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(workload, precision, tile):
    """HBM bytes per update launch from committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None
    when they are missing or were taken on another kernel source or tile."""
    tag = "-".join(str(int(x)) for x in tile)
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}_tile{tag}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha") != _kernel_sha() or list(rec.get("tile", [])) != list(tile):
        return None
    return rec.get("hbm_bytes_per_launch")


# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 FP64 (or non-packed FP32)
# VALU instruction per SIMD every 4 cycles at 2.4 GHz
VALU_PEAK = 1024 * 2.4e9 / 4


def _alu(workload, precision, tile, avg_ms):
    """The update kernel's VALU issue rate: wavefront VALU instructions per
    launch from a committed rocprofv3 counter run (same kernel source and
    tile) over the launch duration timed live, against the issue peak."""
    tag = "-".join(str(int(x)) for x in tile)
    path = os.path.join(ROOT, "profiles", f"valu_{workload}_{precision}_tile{tag}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha") != _kernel_sha():
        return None
    achieved = rec["valu_wave_instr_per_launch"] / (avg_ms * 1e-3)
    return {"achieved": achieved, "peak": VALU_PEAK, "unit": "wave64 VALU instr/s", "frac": achieved / VALU_PEAK,
            "lane_instr_per_update": rec["valu_lane_instr_per_update"], "busy_frac_counter": rec["valu_busy_frac"]}


def copy_ceiling(gib=1.0, reps=5):
    """Practical HBM ceiling: the library's plain streaming copy kernel
    (every byte read once and written once) over two buffers of `gib` GiB,
    timed with HIP events on its stream; GB/s counts read plus written
    bytes, the best of `reps` launches."""
    import torch
    from paper_2512_20252_amd import ibdvm

    n = int(gib * 2 ** 30)
    src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    ibdvm.stream_copy(src, dst, stream)
    best = None
    for _ in range(reps):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        ibdvm.stream_copy(src, dst, stream)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        best = ms if best is None else min(best, ms)
    assert torch.equal(src[:1024], dst[:1024])
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": 2 * n / (best * 1e-3) / 1e9, "bytes_each_way": n, "ms": best,
            "kernel": "k_stream_copy (ibdvm_stream_copy), 16-byte lanes"}


def run_gpu(case, precision, steps, warmup, seed=0, profile=True, tile=None):
    """Warm-up steps, then `steps` eager steps with kernel timing (HIP events
    around each launch on the solve's stream), then the timed region: the
    same number of steps as one replay of a captured graph (an even count;
    an odd count is timed as eager steps), bracketed by events on the
    solve's stream."""
    import torch
    from paper_2512_20252_amd import cases, ibdvm

    stream = torch.cuda.Stream()
    s = ibdvm.Solver(case, precision=precision, stream=stream)
    s.init_freestream(cases.noise(case, seed), 1e-3)
    if tile:
        s.set_tile(*tile)
    else:
        s.autotune(reps=3)
    s.step(warmup)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    prof, ms_eager = None, None
    if profile:
        s.profile(True)
        torch.cuda.synchronize()
        t0.record(stream)
        s.step(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        ms_eager = t0.elapsed_time(t1)
        prof = s.profile_read()
        s.profile(False)
    g = None
    if steps % 2 == 0:
        g = ibdvm.Graph(s, steps)
        g.launch()  # untimed: the first replay uploads the graph
    torch.cuda.synchronize()
    t0.record(stream)
    if g:
        g.launch()
    else:
        s.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    if g:
        g.close()
    _, cd, _, _ = s.surface_forces()
    out = {"ms": ms, "ms_eager": ms_eager, "graph": g is not None, "prof": prof, "cd": cd, "nfluid": s.nfluid,
           "NV": s.NV, "dim": s.dim, "tile": s.get_tile()}
    del s
    torch.cuda.empty_cache()
    return out


def shard_shapes(steps, warmup, full_rate, G=8):
    """The per-GPU shares of the 256^2 cylinder split over G GPUs, each at
    its real shape, for the two ways the step can be split:
    * velocity: the 256^2 cells with 48 x 48/G velocity nodes (the midpoint
      grid of the same box at G times the y spacing, which a share of
      interleaved node rows has); the per-cell moment all-reduce and the
      pairs' all-gather that complete a sharded step are not run;
    * slab: 256 x 256/G cells around the body with the full 48^2 grid;
      freestream rows stand in for the neighbours' halo rows, whose
      exchange is not run.
    Both storage forms, autotuned as the full-grid leg is; each rate per
    update is compared with the full grid's FP64 rate."""
    from paper_2512_20252_amd import cases

    out = {"G": G, "steps": steps, "warmup": warmup}
    shapes = {
        "velocity": (cases.cylinder_256_velocity_shard(G=G),
                     f"256x256 cells, 48x{48 // G} velocity nodes on [-6,6]^2 (stand-in nodes of a share's spacing)",
                     {"allreduce_bytes_per_step": 65536 * 9 * 8}),
        "slab": (cases.cylinder_256_slab(G=G),
                 f"256x{256 // G} cells on [-8,8]x[-{8 / G},{8 / G}] around the body, 48x48 velocity nodes",
                 {"halo_bytes_per_face_per_step": 2 * 256 * 2304 * 2 * 8}),
    }
    for name, (case, desc, comm) in shapes.items():
        o = {"workload": f"per-GPU share of the 256x256 x 48x48 cylinder (Kn 0.1, Ma 0.3) over {G} GPUs: {desc}",
             "not_run": "the exchange between shares", **comm}
        for prec in ("f64", "f32"):
            r = run_gpu(case, prec, steps, warmup)
            upd = r["nfluid"] * r["NV"]
            avg = r["prof"]["update_ms"] / max(r["prof"]["update_launches"], 1)
            o[prec] = {"updates_per_s": upd * steps / (r["ms"] * 1e-3), "ms_per_step": r["ms"] / steps,
                       "update_avg_launch_ms": avg,
                       "hbm_frac": upd * B_ALG[(2, prec)] / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "fill_avg_launch_ms": r["prof"]["fill_ms"] / max(r["prof"]["fill_launches"], 1),
                       "tile": list(r["tile"]), "fluid_cells": r["nfluid"], "velocity_nodes": r["NV"]}
        o["f64_rate_vs_full_grid"] = o["f64"]["updates_per_s"] / full_rate
        out[name] = o
    return out


def sphere3d(n, steps, warmup, tiles):
    """Full-distribution 3D sphere leg (R=0.5 in [-4,4]^3, n^3 cells, 24^3
    velocity nodes on [-6,6]^3, Kn 0.1, Ma 1.5): FP64 and FP32-storage update
    rates, algorithmic HBM bytes per update launch over its HIP-event duration,
    HBM bytes from committed counter runs of the same kernel and tile, and
    the C_D difference of the two forms after the same steps.  The initial
    state is drawn on the device from a counter-based generator (a host array
    of the 96^3 x 24^3 state would be 98 GB)."""
    import torch
    from paper_2512_20252_amd import cases, ibdvm

    case = cases.sphere(n=n, vn=24)
    out = {"workload": f"3D sphere R=0.5 on [-4,4]^3, {n}^3 cells, 24^3 velocity nodes on [-6,6]^3, "
                       "Kn 0.1, Ma 1.5, Shakhov, diffuse wall", "steps": steps, "warmup": warmup}
    for prec in ("f64", "f32"):
        s = ibdvm.Solver(case, precision=prec, stream=torch.cuda.Stream())
        s.init_freestream_hashed(0, 1e-3)
        if tiles[prec]:
            s.set_tile(*tiles[prec])
            tile = s.get_tile()
        else:
            tile = s.autotune(reps=2)
        s.step(warmup)
        s.profile(True)
        t = time.perf_counter()
        s.step(steps)
        _, cd, _, _ = s.surface_forces()
        wall = time.perf_counter() - t
        prof = s.profile_read()
        upd = s.nfluid * s.NV
        avg = prof["update_ms"] / max(prof["update_launches"], 1)
        gbs = upd * B_ALG[(3, prec)] / (avg * 1e-3) / 1e9
        out[prec] = {"updates_per_s": upd * steps / wall, "ms_per_step": wall * 1e3 / steps,
                     "update_avg_launch_ms": avg, "update_GBs_alg": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                     "fill_avg_launch_ms": prof["fill_ms"] / max(prof["fill_launches"], 1), "tile": list(tile),
                     "traffic": _traffic(f"sphere_{n}x{n}x{n}_v24x24x24", prec, tile),
                     "alu": _alu(f"sphere_{n}x{n}x{n}_v24x24x24", prec, tile, avg),
                     "CD": cd, "fluid_cells": s.nfluid, "velocity_nodes": s.NV,
                     "footprint_GB": ibdvm.footprint(case, prec) / 1e9}
        del s
        torch.cuda.empty_cache()
    out["ratio_f32_vs_f64"] = out["f32"]["updates_per_s"] / out["f64"]["updates_per_s"]
    out["dCD_f32_vs_f64"] = abs(out["f32"]["CD"] - out["f64"]["CD"])
    return out


def hypersonic(steps, warmup):
    """Hypersonic bodies leg (the airfoil and the ellipse of the seeded
    draw at Ma 5, Kn 0.05, alpha 0.8 on 512 x 384 cells with 64^2 velocity
    nodes on [-10,10]^2): per body and storage form, updates/s of eager
    steps, update and fill-phase launch times, and C_D."""
    import torch
    from paper_2512_20252_amd import cases, ibdvm

    out = {"workload": "2D airfoil and ellipse at Ma 5, Kn 0.05, alpha 0.8, 512x384 cells, 64x64 velocity nodes "
                       "on [-10,10]^2", "steps": steps, "warmup": warmup}
    out["f32_storage"] = "f itself (IBDVM_FLAG_F32_ABSOLUTE): the wakes empty toward vacuum, where offsets " \
                         "from the freestream Maxwellian would cancel the digits of f"
    for body, case in zip(("airfoil", "ellipse"), cases.hypersonic_bodies(0)):
        case = cases.case(**dict(case, flags=("f32_absolute",)))
        for prec in ("f64", "f32"):
            s = ibdvm.Solver(case, precision=prec)
            s.init_freestream()
            tile = s.autotune(reps=2)
            s.step(warmup)
            torch.cuda.synchronize()
            s.profile(True)
            t = time.perf_counter()
            s.step(steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
            prof = s.profile_read()
            upd = s.nfluid * s.NV
            avg = prof["update_ms"] / max(prof["update_launches"], 1)
            out[f"{body}_{prec}"] = {"updates_per_s": upd * steps / wall, "ms_per_step": wall * 1e3 / steps,
                                     "update_avg_launch_ms": avg,
                                     "hbm_frac": upd * B_ALG[(2, prec)] / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                     "fill_avg_launch_ms": prof["fill_ms"] / max(prof["fill_launches"], 1),
                                     "tile": list(tile), "CD": s.surface_forces()[1], "pairs": s.npairs}
            del s
            torch.cuda.empty_cache()
    return out


def cavity(n, vn, steps, warmup, tiles):
    """Lid-driven cavity leg (unit square, n^2 cells, vn^2 velocity nodes on
    [-5,5]^2, cylinder of diameter 0.25 at the centre, lid 0.15, T_w = 1,
    Kn 0.075, gas initially at rest): FP64 and FP32-storage update rates,
    algorithmic HBM bytes per update launch over its HIP-event duration, and
    the fill phase (immersed-boundary ghosts plus the outer-wall ghost rows)
    per step."""
    import torch
    from paper_2512_20252_amd import cases, ibdvm

    case = cases.cavity(n=n, vn=vn)
    out = {"workload": f"2D lid-driven cavity with a cylinder (D=0.25), {n}^2 cells, {vn}^2 velocity nodes on "
                       "[-5,5]^2, lid 0.15, T_w 1, Kn 0.075, diffuse outer walls", "steps": steps, "warmup": warmup}
    for prec in ("f64", "f32"):
        s = ibdvm.Solver(case, precision=prec)
        s.init_freestream()
        if tiles[prec]:
            s.set_tile(*tiles[prec])
            tile = s.get_tile()
        else:
            tile = s.autotune(reps=2)
        s.step(warmup)
        torch.cuda.synchronize()
        s.profile(True)
        t = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        prof = s.profile_read()
        upd = s.nfluid * s.NV
        avg = prof["update_ms"] / max(prof["update_launches"], 1)
        gbs = upd * B_ALG[(2, prec)] / (avg * 1e-3) / 1e9
        m = s.moments()
        out[prec] = {"updates_per_s": upd * steps / wall, "ms_per_step": wall * 1e3 / steps,
                     "update_avg_launch_ms": avg, "update_GBs_alg": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                     "fill_avg_launch_ms": prof["fill_ms"] / max(prof["fill_launches"], 1), "tile": list(tile),
                     "lid_row_mean_Ux": float(m[-n:, 1].mean()), "fluid_cells": s.nfluid, "velocity_nodes": s.NV}
        del s
        torch.cuda.empty_cache()
    out["ratio_f32_vs_f64"] = out["f32"]["updates_per_s"] / out["f64"]["updates_per_s"]
    return out


def implicit_collision(Kn, steps, warmup):
    """Semi-implicit collision leg: the 256^2 cylinder (48^2 nodes, Ma 0.3)
    at a small Knudsen number, FP64, with the explicit step and with the
    semi-implicit collision: time step, wall time per step, simulated time
    per wall second, update and fill-phase launch times (the fill phase
    includes the moment finish, which does the implicit relaxation)."""
    import torch
    from paper_2512_20252_amd import cases, ibdvm

    out = {"workload": f"2D cylinder R=0.5 on [-8,8]^2, 256x256 cells, 48x48 velocity nodes on [-6,6]^2, "
                       f"Kn {Kn}, Ma 0.3, FP64", "steps": steps, "warmup": warmup}
    for mode, flags in (("explicit", ()), ("implicit", ("implicit",))):
        case = cases.case(**dict(cases.cylinder_256(Kn=Kn, Ma=0.3), flags=flags))
        s = ibdvm.Solver(case)
        s.init_freestream(cases.noise(case, 0), 1e-3)
        tile = s.autotune(reps=2)
        s.step(warmup)
        torch.cuda.synchronize()
        s.profile(True)
        t0 = s.clock()["time"]
        t = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        prof = s.profile_read()
        clk = s.clock()
        out[mode] = {"dt": clk["dt"], "ms_per_step": wall * 1e3 / steps,
                     "sim_time_per_s": (clk["time"] - t0) / wall,
                     "updates_per_s": s.nfluid * s.NV * steps / wall,
                     "update_avg_launch_ms": prof["update_ms"] / max(prof["update_launches"], 1),
                     "fill_ms_per_step": prof["fill_ms"] / steps, "tile": list(tile)}
        del s
        torch.cuda.empty_cache()
    out["dt_ratio"] = out["implicit"]["dt"] / out["explicit"]["dt"]
    out["sim_time_rate_ratio"] = out["implicit"]["sim_time_per_s"] / out["explicit"]["sim_time_per_s"]
    return out


def _steady(case, t_end, tag, block=1000, precision="f64"):
    """Run a solve from its freestream (rest for Ma 0) to time t_end in
    replays of a captured graph of `block` steps; moments, wall points,
    step count, last residual and wall time."""
    import torch
    from paper_2512_20252_amd import ibdvm

    s = ibdvm.Solver(case, precision=precision, stream=torch.cuda.Stream())
    s.init_freestream()
    g = ibdvm.Graph(s, block)
    t0, k = time.perf_counter(), 0
    last = t0
    try:
        while s.clock()["time"] < t_end:
            g.launch()
            k += 1
            if time.perf_counter() - last > 20.0:
                last = time.perf_counter()
                print(f"{tag}: t = {s.clock()['time']:.1f}", file=sys.stderr, flush=True)
        s.step(2)
        r = {"m": s.moments(), "wall": s.surface_forces(), "steps": s.clock()["step"],
             "residual": s.residual()[1], "seconds": time.perf_counter() - t0}
        print(f"{tag}: {r['steps']} steps in {r['seconds']:.1f} s", file=sys.stderr, flush=True)
    except ibdvm.IbdvmError as e:
        # the device health word reported a non-physical state; the solve is unusable from here
        r = {"failed": str(e), "steps_launched": k * block}
        print(f"{tag}: failed after at most {k * block} steps: {e}", file=sys.stderr, flush=True)
    g.close()
    s.close()
    torch.cuda.empty_cache()
    return r


def slip_study(n, t_end, modes=6, block=500):
    """Wall slip of the hypersonic cylinder (the Section 4 comparison of the
    slip velocity along the wall with and without the upwind-weighted
    interpolation): R = 1 at Ma 5, Kn 0.1, T_w = 1 on a uniform n x n grid
    of [-6,10] x [-8,8] with 60^2 velocity nodes on [-10,10]^2, run to time
    t_end with the upwind weights of Section 3.2.2, with uniform weights
    (NO_UPWIND) and with the naive axis extrapolation of Section 3.3.3.  Per
    run: the tangential slip velocity u_s . t of the wall gas at every wall
    point (t anticlockwise), and the zigzag amplitude: the RMS residual of a
    least-squares fit of u_s . t by Fourier modes up to `modes` in the polar
    angle, relative to the largest |u_s . t|."""
    import numpy as np
    import torch
    from paper_2512_20252_amd import cases, ibdvm

    base = cases.case(dim=2, n=(n, n), lo=(-6.0, -8.0), hi=(10.0, 8.0), vn=(60, 60), vlo=(-10.0, -10.0),
                      vhi=(10.0, 10.0), geometry="circle", size=(1.0, 0.0, 0.0), Kn=0.1, Ma=5.0)
    out = {"workload": f"2D cylinder R=1 at Ma 5, Kn 0.1, T_w 1, {n}x{n} cells on [-6,10]x[-8,8], 60^2 velocity "
                       f"nodes on [-10,10]^2, to t = {t_end}", "modes": modes}
    for tag, flags in (("upwind", ()), ("uniform_weights", ("no_upwind",)), ("naive", ("naive",))):
        c = cases.case(**dict(base, flags=flags))
        s = ibdvm.Solver(c, stream=torch.cuda.Stream())
        s.init_freestream()
        g = ibdvm.Graph(s, block)
        r, done = {"status": "ok"}, 0
        try:
            while s.clock()["time"] < t_end:
                g.launch()
                done += block
            _, cd, _, w = s.surface_forces()
            xw, nw, us = w[:, 0:2], w[:, 3:5], w[:, 14:16]
            tang = np.stack([-nw[:, 1], nw[:, 0]], 1)
            ut = np.sum(us * tang, axis=1)
            th = np.arctan2(xw[:, 1], xw[:, 0])
            cols = [np.ones_like(th)] + [f(k * th) for k in range(1, modes + 1) for f in (np.cos, np.sin)]
            Amat = np.stack(cols, 1)
            coef, *_ = np.linalg.lstsq(Amat, ut, rcond=None)
            resid = ut - Amat @ coef
            order = np.argsort(th)
            r.update({"CD": cd, "steps": s.clock()["step"], "wall_points": int(len(ut)),
                      "max_abs_slip": float(np.max(np.abs(ut))),
                      "zigzag_rms_rel": float(np.sqrt(np.mean(resid ** 2)) / np.max(np.abs(ut))),
                      "theta": [round(float(x), 4) for x in th[order]],
                      "slip": [round(float(x), 5) for x in ut[order]]})
        except ibdvm.IbdvmError as e:
            # an unstable context answers every later call with IBDVM_E_STATE
            r = {"status": f"failed: {e}", "steps_launched": done}
        g.close()
        s.close()
        torch.cuda.empty_cache()
        out[tag] = r
        print(f"slip study: {tag}: {r.get('zigzag_rms_rel', r['status'])}", file=sys.stderr, flush=True)
    return out


def _l1(a, b):
    import numpy as np
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


def space_study(levels, nref, Kn, Ma, vn, t_end, block=500):
    """Physical-space convergence (the order estimates of Section 3.3: wall
    discontinuities cost O(dx^2) in the moments while dx is above about
    lambda^2 / R_w, O(dx^(3/2)) below it): the cylinder R = 0.5 on
    [-4,4]^2 at Kn, Ma on levels^2 cells, each run to t_end on the same
    vn^2 velocity grid on [-6,6]^2, against an nref^2 run.  Errors: C_D
    relative; p_w, the tangential shear tau_w . t and q_n along the wall,
    each wall point against the reference's profile interpolated at its
    polar angle (L1 relative); rho and T over the fluid cells, the
    reference averaged over the (nref/n)^2 fine cells of each coarse cell
    (blocks that touch the body in either grid left out).  Observed orders
    are least-squares slopes against dx."""
    import numpy as np
    from paper_2512_20252_amd import cases

    def case(n):
        return cases.case(dim=2, n=(n, n), lo=(-4.0, -4.0), hi=(4.0, 4.0), vn=(vn, vn), vlo=(-6.0, -6.0),
                          vhi=(6.0, 6.0), geometry="circle", size=(0.5, 0.0, 0.0), Kn=Kn, Ma=Ma)

    def wall_profile(w):
        th = np.arctan2(w[:, 1], w[:, 0])
        tau_t = -w[:, 4] * w[:, 8] + w[:, 3] * w[:, 9]  # tau_w . t with t = (-n_y, n_x)
        o = np.argsort(th)
        return th[o], {"p_w": w[o, 7], "tau_w": tau_t[o], "q_n": w[o, 11]}

    ref = _steady(case(nref), t_end, f"space study reference {nref}^2", block)
    th_ref, W_ref = wall_profile(ref["wall"][3])
    M_ref = ref["m"].reshape(nref, nref, 8)
    out = {"workload": f"2D cylinder R=0.5 on [-4,4]^2 at Kn {Kn}, Ma {Ma}, {vn}^2 velocity nodes on [-6,6]^2, "
                       f"cells {'/'.join(str(v) for v in levels)} squared against {nref}^2, t = {t_end}",
           "reference": {"CD": ref["wall"][1], "steps": ref["steps"], "seconds": ref["seconds"]}, "levels": {}}
    for n in levels:
        r = _steady(case(n), t_end, f"space study {n}^2", block)
        th, W = wall_profile(r["wall"][3])
        e = {"CD": abs(r["wall"][1] - ref["wall"][1]) / abs(ref["wall"][1]), "steps": r["steps"]}
        for k in W:
            vref = np.interp(th, th_ref, W_ref[k], period=2 * np.pi)
            e[k] = float(np.sum(np.abs(W[k] - vref)) / np.sum(np.abs(vref)))
        k = nref // n
        fine = M_ref.reshape(n, k, n, k, 8)
        coarse = r["m"].reshape(n, n, 8)
        ok = np.isfinite(fine[..., 0]).all(axis=(1, 3)) & np.isfinite(coarse[..., 0])
        for j, name in ((0, "rho"), (4, "T")):
            avg = fine[..., j].mean(axis=(1, 3))
            e[name] = float(np.sum(np.abs(coarse[ok, j] - avg[ok])) / np.sum(np.abs(avg[ok])))
        out["levels"][str(n)] = e
    dx = np.array([8.0 / n for n in levels])
    out["observed_order"] = {}
    for q in ("CD", "p_w", "tau_w", "q_n", "rho", "T"):
        err = np.array([out["levels"][str(n)][q] for n in levels])
        if np.all(err > 0):
            out["observed_order"][q] = float(np.polyfit(np.log(dx), np.log(err), 1)[0])
    return out


def vmesh_study(levels, nref, t_end, beta):
    """Velocity-mesh efficiency: the 32^2 cylinder (Ma 0.5, Kn 0.1) at steady
    state (t = t_end) on uniform midpoint and stretched (R31, beta) velocity
    grids of levels^2 nodes on [-5,5]^2, with dual-cell and with Jacobian
    weights (R36), against a uniform nref^2 reference:
    relative errors of C_D and L1 errors of p_w, tau_w and q_n over the wall
    points.  Same N means the same cost per step."""
    import numpy as np
    from paper_2512_20252_amd import cases

    base = dict(cases.cylinder_small(), rule="midpoint")
    ref = _steady(cases.case(**dict(base, vn=(nref, nref))), t_end, f"vmesh reference {nref}^2")
    cd_ref, W = ref["wall"][1], ref["wall"][3]
    out = {"workload": f"2D cylinder 32^2 cells (R=0.3, Ma 0.5, Kn 0.1), velocity grids "
                       f"{'/'.join(str(v) for v in levels)} squared on [-5,5]^2, uniform midpoint and stretched "
                       f"(beta {beta}), against uniform {nref}^2, steady state (t = {t_end})",
           "reference": {"CD": cd_ref, "steps": ref["steps"], "residual": ref["residual"]}}
    for tag, extra in (("uniform", {}), ("stretched", {"rule": "stretched", "vstretch": beta}),
                       ("stretched_jacobian", {"rule": "stretched", "vstretch": beta, "vweights": "jacobian"})):
        errs = {}
        for vn in levels:
            r = _steady(cases.case(**dict(base, vn=(vn, vn), **extra)), t_end, f"vmesh {tag} {vn}^2")
            w = r["wall"][3]
            errs[str(vn)] = {"CD": abs(r["wall"][1] - cd_ref) / abs(cd_ref), "p_w": _l1(w[:, 7], W[:, 7]),
                             "tau_w": _l1(w[:, 8:10], W[:, 8:10]), "q_n": _l1(w[:, 11], W[:, 11]),
                             "steps": r["steps"]}
        out[tag] = errs
    return out


def refined_study(levels, nref, n, t_end, amp, width, shapes=None):
    """Locally refined velocity grid (R35) against uniform grids on the
    hypersonic cylinder, where the freestream Maxwellian (centred at
    U_inf = 4.56) and the wall Maxwellian (centred at 0) are narrow against
    the [-10,10]^2 velocity box (the reason for the paper's refined sphere
    mesh in Section 4): R = 1 at Ma 5, Kn 0.1, T_w = 1 on n x n cells of
    [-6,10] x [-8,8], steady state at t_end; velocity grids of levels^2
    nodes, uniform midpoint and refined (density 1 + amp(exp(-(x/w)^2) +
    exp(-((x - U_inf)/w)^2)) on x, one bump at 0 on y) with dual-cell weights
    (R35) and with the map's derivative as weight (R36), against a uniform
    nref^2 reference.  Relative C_D error and L1 errors of p_w, tau_w and q_n
    over the wall points; the same N costs the same per step."""
    from paper_2512_20252_amd import cases

    uinf = 5.0 * (5.0 / 6.0) ** 0.5
    base = cases.case(dim=2, n=(n, n), lo=(-6.0, -8.0), hi=(10.0, 8.0), vlo=(-10.0, -10.0), vhi=(10.0, 10.0),
                      geometry="circle", size=(1.0, 0.0, 0.0), Kn=0.1, Ma=5.0)
    ref = _steady(cases.case(**dict(base, vn=(nref, nref))), t_end, f"refined study reference {nref}^2", 500)
    cd_ref, W = ref["wall"][1], ref["wall"][3]
    out = {"workload": f"2D cylinder R=1 at Ma 5, Kn 0.1, {n}^2 cells on [-6,10]x[-8,8], velocity grids "
                       f"{'/'.join(str(v) for v in levels)} squared on [-10,10]^2, uniform and refined (amp {amp}, "
                       f"width {width}, centres 0 and U_inf on x), against uniform {nref}^2, t = {t_end}",
           "reference": {"CD": cd_ref, "steps": ref["steps"]}}
    runs = [("uniform", {})] + [(f"refined_A{a}_w{w}" + ("_jacobian" if wt == "jacobian" else ""),
                                 {"rule": "refined", "vref_amp": a, "vref_width": w, "vref_centre": (uinf, 0.0, 0.0),
                                  "vweights": wt})
                                for wt in ("cell", "jacobian") for a, w in (shapes or [(amp, width)])]
    for tag, extra in runs:
        errs = {}
        for vn in levels:
            r = _steady(cases.case(**dict(base, vn=(vn, vn), **extra)), t_end, f"refined study {tag} {vn}^2", 500)
            if "failed" in r:
                errs[str(vn)] = {"failed": r["failed"], "steps_launched": r["steps_launched"]}
                continue
            w = r["wall"][3]
            errs[str(vn)] = {"CD": abs(r["wall"][1] - cd_ref) / abs(cd_ref), "p_w": _l1(w[:, 7], W[:, 7]),
                             "tau_w": _l1(w[:, 8:10], W[:, 8:10]), "q_n": _l1(w[:, 11], W[:, 11]),
                             "steps": r["steps"]}
        out[tag] = errs
    return out


def sphere_vmesh_study(n, levels, nref, t_end, amp, width, block=200):
    """Velocity meshes of the Section 4 sphere: Ma 3.834, wall at the
    stagnation temperature T_w = 1 + (gamma - 1) Ma^2 / 2, velocity box
    [-3 sqrt(T_w), 3 sqrt(T_w)]^3, here at Kn 0.1 on n^3 cells of [-4,4]^3
    (R = 0.5), FP32 storage of f; uniform midpoint grids of levels^3 nodes
    and refined grids with the map's derivative (R36) or the dual-cell
    widths (R35) as weights (density
    1 + amp(exp(-(x/w)^2) + exp(-((x - U_inf)/w)^2)) on x, one bump at 0 on
    y and z), against a uniform nref^3 reference, each run to time t_end.
    Relative C_D error and L1 errors of p_w, tau_w and q_n over the wall
    points."""
    from paper_2512_20252_amd import cases

    Ma, gam = 3.834, 5.0 / 3.0
    Tw = 1.0 + 0.5 * (gam - 1.0) * Ma * Ma
    V = 3.0 * Tw ** 0.5
    uinf = Ma * (gam / 2.0) ** 0.5
    base = cases.case(**dict(cases.sphere(n=n, vn=nref), Ma=Ma, Tw=Tw, vlo=(-V,) * 3, vhi=(V,) * 3))

    def run(vn, extra, tag):
        return _steady(cases.case(**dict(base, vn=(vn,) * 3, **extra)), t_end, tag, block, precision="f32")

    ref = run(nref, {}, f"sphere study reference {nref}^3")
    cd_ref, W = ref["wall"][1], ref["wall"][3]
    out = {"workload": f"3D sphere R=0.5 at Ma {Ma}, Kn 0.1, T_w {Tw:.3f}, {n}^3 cells on [-4,4]^3, velocity box "
                       f"[-{V:.3f},{V:.3f}]^3, uniform and refined (amp {amp}, width {width}, Jacobian or cell weights) grids "
                       f"of {'/'.join(str(v) for v in levels)} cubed against uniform {nref}^3, FP32 storage of f, "
                       f"t = {t_end}",
           "reference": {"CD": cd_ref, "steps": ref["steps"], "seconds": ref["seconds"]}}
    refined = {"rule": "refined", "vref_amp": amp, "vref_width": width, "vref_centre": (uinf, 0.0, 0.0)}
    for tag, extra in (("uniform", {}), ("refined_jacobian", dict(refined, vweights="jacobian")),
                       ("refined_cell", dict(refined, vweights="cell"))):
        errs = {}
        for vn in levels:
            r = run(vn, extra, f"sphere study {tag} {vn}^3")
            if "failed" in r:
                errs[str(vn)] = {"failed": r["failed"], "steps_launched": r["steps_launched"]}
                continue
            w = r["wall"][3]
            errs[str(vn)] = {"CD": abs(r["wall"][1] - cd_ref) / abs(cd_ref), "p_w": _l1(w[:, 7], W[:, 7]),
                             "tau_w": _l1(w[:, 8:11], W[:, 8:11]), "q_n": _l1(w[:, 11], W[:, 11]),
                             "steps": r["steps"], "seconds": r["seconds"]}
        out[tag] = errs
    return out


def cavity_velocity_study(n, levels, nref, t_end, block=1000):
    """Velocity-space convergence of the lid-driven cavity at steady state
    (the study of Section 4): the cavity on n^2 cells with velocity meshes
    levels^2, with and without the cut-cell correction, each run from rest
    to time t_end (past the point where the residual stops falling), against
    a reference on nref^2 nodes with the correction.  L1 errors relative to
    the reference: rho, |U| and T over the fluid cells, p_w, tau_w, q_n and
    the gas temperature T_s and slip velocity u_s at the wall points;
    observed orders are least-squares slopes of log error against log N."""
    import numpy as np
    from paper_2512_20252_amd import cases

    def steady(vn, flags):
        r = _steady(cases.case(**dict(cases.cavity(n=n, vn=vn), flags=flags)), t_end,
                    f"cavity study {vn}^2 {'/'.join(flags)}", block)
        r["wall"] = r["wall"][3]
        return r

    l1 = _l1
    ref = steady(nref, ())
    ok = np.isfinite(ref["m"][:, 0])
    M, W = ref["m"][ok], ref["wall"]
    out = {"workload": f"2D lid-driven cavity with a cylinder, {n}^2 cells, velocity meshes "
                       f"{'/'.join(str(v) for v in levels)} squared against {nref}^2 on [-5,5]^2, steady state (t = {t_end})",
           "reference": {"steps": ref["steps"], "residual": ref["residual"], "seconds": ref["seconds"]}}
    for tag, flags in (("cutcell", ()), ("no_cutcell", ("no_cutcell",))):
        errs = {}
        for vn in levels:
            r = steady(vn, flags)
            m, w = r["m"][ok], r["wall"]
            errs[vn] = {"rho": l1(m[:, 0], M[:, 0]),
                        "U": float(np.sum(np.linalg.norm(m[:, 1:3] - M[:, 1:3], axis=1)) /
                                   np.sum(np.linalg.norm(M[:, 1:3], axis=1))),
                        "T": l1(m[:, 4], M[:, 4]), "p_w": l1(w[:, 7], W[:, 7]), "tau_w": l1(w[:, 8:10], W[:, 8:10]),
                        "q_n": l1(w[:, 11], W[:, 11]), "T_s": l1(w[:, 13], W[:, 13]),
                        "u_s": l1(w[:, 14:16], W[:, 14:16]), "steps": r["steps"], "residual": r["residual"]}
        ln = np.log(np.array(levels, float))
        orders = {q: float(-np.polyfit(ln, np.log([errs[v][q] for v in levels]), 1)[0])
                  for q in ("rho", "U", "T", "p_w", "tau_w", "q_n", "T_s", "u_s")}
        out[tag] = {"L1": {str(v): e for v, e in errs.items()}, "orders": orders}
    return out


def precision_sweep(cases_kn_ma, rtol, cap, block=100, sphere_n=48, hypersonic=False, atol=None):
    """FP32 storage against FP64 over the 256^2 cylinder's Kn x Ma sweep, a
    sphere of sphere_n^3 cells (24^3 nodes, Kn 0.1, Ma 1.5) and, with
    `hypersonic`, the Ma-5 airfoil and ellipse at full size (512 x 384 cells,
    64^2 nodes, FP32 storing f itself): the cylinders from the seed-0
    perturbation, the sphere from the hashed one, the bodies from the
    freestream, in replays of a captured graph of `block` steps; the FP64
    form runs until C_D changes by less than rtol relative (or, given atol,
    by less than atol) over a replay, or `cap` steps, the FP32 form then
    runs the same number of steps, so the two C_D differ by precision only;
    the updates/s of each form over its run."""
    import torch
    from paper_2512_20252_amd import cases, ibdvm

    parts = []
    if cases_kn_ma:
        parts.append("2D cylinder R=0.5 on [-8,8]^2, 256x256 cells, 48x48 velocity nodes on [-6,6]^2")
    if sphere_n:
        parts.append(f"3D sphere on {sphere_n}^3 cells, 24^3 nodes")
    if hypersonic:
        parts.append("2D airfoil and ellipse at Ma 5, Kn 0.05, alpha 0.8, 512x384 cells, 64x64 nodes on [-10,10]^2")
    crit = f"{atol:g} absolute" if atol is not None else f"{rtol:g} relative"
    out = {"workload": "; ".join(parts) + f"; C_D change below {crit} per {block} steps or {cap} steps",
           "cases": []}
    runs = [(f"cylinder Kn {Kn} Ma {Ma}", {"Kn": Kn, "Ma": Ma}, cases.cylinder_256(Kn=Kn, Ma=Ma))
            for Kn, Ma in cases_kn_ma]
    if sphere_n:
        runs.append((f"sphere {sphere_n}^3", {"sphere_n": sphere_n, "Kn": 0.1, "Ma": 1.5},
                     cases.sphere(n=sphere_n, vn=24)))
    if hypersonic:
        for body, case in zip(("airfoil", "ellipse"), cases.hypersonic_bodies(0)):
            runs.append((f"hypersonic {body}", {"body": body, "Kn": 0.05, "Ma": 5.0, "alpha": 0.8},
                         cases.case(**dict(case, flags=("f32_absolute",)))))
    tol = atol if atol is not None else rtol
    for label, row, case in runs:
        row = dict(row)
        for prec in ("f64", "f32"):
            if prec == "f32" and row["f64"]["failed"]:
                break
            s = ibdvm.Solver(case, precision=prec, stream=torch.cuda.Stream())
            if "body" in row:
                s.init_freestream()
                row[prec + "_tile"] = list(s.autotune(reps=2))
            elif case["dim"] == 2:
                s.init_freestream(cases.noise(case, 0), 1e-3)
                s.set_tile(2, 4, 32)
            else:
                s.init_freestream_hashed(0, 1e-3)  # a host array of the 3D state would be large
            g = ibdvm.Graph(s, block)
            cd_prev, change, steps, t = None, None, 0, time.perf_counter()
            t_print = t
            limit = cap if prec == "f64" else row["f64"]["steps"]
            cd, failed = None, None
            try:
                while steps < limit:
                    g.launch()
                    steps += block
                    cd = s.surface_forces()[1]
                    change = None if cd_prev is None else (abs(cd - cd_prev) if atol is not None
                                                           else abs(cd - cd_prev) / abs(cd))
                    cd_prev = cd
                    if time.perf_counter() - t_print > 30.0:
                        t_print = time.perf_counter()
                        print(f"precision sweep: {label} {prec}: step {steps}, C_D {cd:.8f}", file=sys.stderr,
                              flush=True)
                    if prec == "f64" and change is not None and change < tol:
                        break
            except ibdvm.IbdvmError as e:  # the health word reported a non-physical state
                failed = f"{e} in the replay ending at step {steps}"
            wall = time.perf_counter() - t
            # the change over the last replay, taken before cd_prev moved on
            row[prec] = {"CD": cd, "steps": steps, "converged": failed is None and change is not None and change < tol,
                         "last_change": change, "updates_per_s": s.nfluid * s.NV * steps / wall, "failed": failed}
            print(f"precision sweep: {label} {prec}: C_D {cd} after {steps} steps" + (f" ({failed})" if failed else ""),
                  file=sys.stderr, flush=True)
            g.close()
            s.close()
            torch.cuda.empty_cache()
        if "f32" in row and not row["f64"]["failed"] and not row["f32"]["failed"]:
            row["dCD"] = abs(row["f32"]["CD"] - row["f64"]["CD"])
            row["dCD_rel"] = row["dCD"] / abs(row["f64"]["CD"])
            row["ratio_f32_vs_f64"] = row["f32"]["updates_per_s"] / row["f64"]["updates_per_s"]
        out["cases"].append(row)
    return out


def fixed_cd_error(block=100):
    """FP32 storage against FP64 at a fixed C_D error: the cylinder's Kn x Ma
    sweep at the 64^2 x 24^2 reduction, each case run on the GPU in both
    forms for the step count at which the FP64 oracle's C_D had converged
    (|dC_D| < 1e-6 |C_D| per 100 steps, or its 10000-step cap), against the
    oracle's C_D stored in tests/golden by a script that runs only the
    oracle."""
    import torch
    from paper_2512_20252_amd import cases, ibdvm

    path = os.path.join(ROOT, "tests", "golden", "converged_cd_cylinder_64x64_v24x24.json")
    if not os.path.exists(path):
        return None
    rows = json.load(open(path))["rows"]
    out = {"workload": "2D cylinder R=0.5 on [-8,8]^2, 64x64 cells, 24x24 velocity nodes on [-6,6]^2, "
                       "Kn {0.01,0.1,1} x Ma {0.3,2}, to the oracle's converged step count",
           "reference": "FP64 CPU oracle, converged C_D (tests/golden/converged_cd_cylinder_64x64_v24x24.json)",
           "cases": []}
    for row in rows:
        c = cases.cylinder_256(Kn=row["Kn"], Ma=row["Ma"], n=64, vn=24)
        u = cases.noise(c, row["seed"])
        r = {"Kn": row["Kn"], "Ma": row["Ma"], "steps": row["steps"], "CD_oracle": row["C_D"]}
        for prec in ("f64", "f32"):
            s = ibdvm.Solver(c, precision=prec, stream=torch.cuda.Stream())
            s.init_freestream(u, 1e-3)
            g = ibdvm.Graph(s, block)
            t = time.perf_counter()
            for _ in range(row["steps"] // block):
                g.launch()
            s.step(row["steps"] % block)
            cd = s.surface_forces()[1]
            r[prec] = {"CD": cd, "dCD_vs_oracle": abs(cd - row["C_D"]), "seconds": time.perf_counter() - t}
            g.close()
            s.close()
        out["cases"].append(r)
    out["max_dCD_f64_vs_oracle"] = max(r["f64"]["dCD_vs_oracle"] for r in out["cases"])
    out["max_dCD_f32_vs_oracle"] = max(r["f32"]["dCD_vs_oracle"] for r in out["cases"])
    return out


def cpu_baseline(case, seed=0):
    """The FP64 oracle on this host: one step of the full workload on all
    its OpenMP threads, and one step of a 128^2-cell window of the same
    workload (the same cell size, body and velocity grid on [-4,4]^2) on one
    thread, each as cell-velocity updates per second."""
    from oracle import oracle as oracle_mod
    from paper_2512_20252_amd import cases

    o = oracle_mod.Oracle(case)
    o.init_freestream(cases.noise(case, seed), 1e-3)
    t = time.perf_counter()
    o.step(1)
    dt = time.perf_counter() - t
    out = {"value": o.nfluid * o.NV / dt, "unit": "cell*vel updates/s", "cores": oracle_mod.threads(),
           "kind": "oracle", "sample": "1 step of the same 256x256 x 48x48 workload (all fluid cells), "
                                       "OpenMP over cells, sequential velocity sums", "seconds": dt}
    del o
    window = cases.case(**dict(case, n=(128, 128), lo=(-4.0, -4.0), hi=(4.0, 4.0)))
    nthreads = oracle_mod.threads()
    oracle_mod.set_threads(1)
    try:
        o = oracle_mod.Oracle(window)
        o.init_freestream(cases.noise(window, seed), 1e-3)
        t = time.perf_counter()
        o.step(1)
        dt1 = time.perf_counter() - t
        out["one_thread"] = {"value": o.nfluid * o.NV / dt1, "cores": oracle_mod.threads(), "seconds": dt1,
                             "sample": "1 step of the 128x128-cell window [-4,4]^2 of the workload (same cell "
                                       "size, body and 48x48 velocity grid)"}
    finally:
        oracle_mod.set_threads(nthreads)
    return out


def serving(nreq, cap, tol, gap_s, max_active=8, seed=0, min_p99=20):
    """Continuous-batching leg: a seeded Poisson stream of mixed 2D solves
    (FP32 storage; f itself for Ma > 2, whose wakes empty toward vacuum)
    through one server; a request converges when C_D changes by less than
    tol relative over a replay of 100 steps, or stops at the step cap.
    Time-to-converged-C_D percentiles with their sample counts (p99 only
    from at least min_p99 samples), the converged fraction and aggregate
    updates/s."""
    import numpy as np
    import torch
    from paper_2512_20252_amd import cases, ibdvm

    reqs, gaps = cases.serving_requests(nreq, seed)
    arrivals = np.cumsum(gaps) * gap_s
    fps = [ibdvm.footprint(c, "f32") for c in reqs]
    free, _ = torch.cuda.mem_get_info()
    ws = int(max(max(fps) + (1 << 20), min(sum(fps) + (1 << 20), 0.8 * free)))
    srv = ibdvm.Server(ws, max_active=max_active, steps_per_replay=100)
    t0, sub, done, samples, index = srv.clock(), 0, [], [], {}
    while len(done) < nreq:
        now = srv.clock() - t0
        while sub < nreq and arrivals[sub] <= now:
            rq = reqs[sub]
            if rq["Ma"] > 2.0:
                rq = cases.case(**dict(rq, flags=("f32_absolute",)))
            index[srv.submit(rq, "f32", seed=sub, amp=1e-3, tol=tol, max_steps=cap)] = sub
            sub += 1
        new = srv.poll(block=False)
        for r in new:
            print(f"serving: request {r['id']} finished after {r['steps']} steps "
                  f"({len(done) + 1}/{nreq})", file=sys.stderr, flush=True)
            done.append(r)
        samples.append(srv.info()["active"])
        time.sleep(0.002)
    srv.close()
    lat = np.array([r["t_done"] - r["t_submit"] for r in done])
    conv = np.array([r["converged"] == 1 for r in done])
    ups = sum(r["updates"] for r in done) / (max(r["t_done"] for r in done) - min(r["t_submit"] for r in done))
    ok = np.array([r["status"] == 0 for r in done])
    pct = lambda x, q, m=1: float(np.percentile(x, q)) if len(x) >= m else None
    return {"requests": nreq, "precision": "f32", "step_cap": cap,
            "criterion": f"|C_D(n) - C_D(n-100)| < {tol:g} |C_D(n)|", "rel_tol_dCD_per_100_steps": tol,
            "mean_arrival_gap_s": gap_s, "max_active": max_active, "workspace_GiB": ws / 2 ** 30,
            "converged": int(conv.sum()), "converged_fraction": float(conv.mean()),
            "capped": int((~conv & ok).sum()), "failed": int((~ok).sum()),
            "p50_time_to_converged_s": pct(lat[conv], 50), "p99_time_to_converged_s": pct(lat[conv], 99, min_p99),
            "n_time_to_converged": int(conv.sum()), "p99_min_samples": min_p99,
            "p50_time_to_done_s": pct(lat, 50), "p99_time_to_done_s": pct(lat, 99, min_p99), "n_time_to_done": len(lat),
            "mean_active": float(np.mean(samples)), "aggregate_updates_per_s": ups,
            "steps": [int(r["steps"]) for r in done],
            "failures": [{"request": index[r["id"]], "status": int(r["status"]), "steps": int(r["steps"]),
                          **{k: reqs[index[r["id"]]][k] for k in ("n", "vn", "geometry", "size", "Kn", "Ma", "alpha")}}
                         for r in done if r["status"] != 0]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--no-f64", action="store_true", help="time only the FP32-storage form")
    ap.add_argument("--tile", type=str, default="", help="V,TX,LY of the FP64 2D update (default: autotune)")
    ap.add_argument("--tile32", type=str, default="", help="V,TX,LY of the FP32-storage 2D update (default: autotune)")
    ap.add_argument("--serving", type=int, default=128,
                    help="requests of the seeded serving stream in the serving leg (0: skip)")
    ap.add_argument("--serving-cap", type=int, default=10000, help="step cap per serving request")
    ap.add_argument("--serving-gap", type=float, default=0.5, help="mean arrival gap of the serving stream, seconds")
    ap.add_argument("--serving-tol", type=float, default=1e-3,
                    help="relative C_D change per 100 steps below which a serving request has converged")
    ap.add_argument("--shard-steps", type=int, default=100,
                    help="timed steps of the per-GPU share shapes of the 256^2 cylinder (0: skip)")
    ap.add_argument("--sphere", type=int, default=96, help="cells per side of the 3D sphere leg (0: skip)")
    ap.add_argument("--sphere-steps", type=int, default=10)
    ap.add_argument("--sphere-tile", type=str, default="1,8,256", help="V,TX,LY of the FP64 3D update ('' to autotune)")
    ap.add_argument("--sphere-tile32", type=str, default="2,16,256", help="V,TX,LY of the FP32 3D update")
    ap.add_argument("--hypersonic-steps", type=int, default=20, help="timed steps of the hypersonic bodies leg (0: skip)")
    ap.add_argument("--cavity", type=int, default=256, help="cells per side of the lid-driven cavity leg (0: skip)")
    ap.add_argument("--cavity-vn", type=int, default=100, help="velocity nodes per axis of the cavity leg")
    ap.add_argument("--cavity-steps", type=int, default=20)
    ap.add_argument("--implicit-kn", type=float, default=2e-4,
                    help="Knudsen number of the semi-implicit collision leg (0: skip)")
    ap.add_argument("--no-fixed-cd", action="store_true",
                    help="skip the converged-C_D comparison of both forms with the oracle (64^2 x 24^2 sweep)")
    ap.add_argument("--precision-sweep", action="store_true",
                    help="add FP32 storage against FP64 over the cylinder's Kn x Ma sweep, run toward convergence")
    ap.add_argument("--sweep-sphere-only", action="store_true", help="run only the sphere case of the precision sweep")
    ap.add_argument("--hypersonic-sweep", action="store_true",
                    help="FP32 storage against FP64 on the Ma-5 airfoil and ellipse at full size, to converged C_D")
    ap.add_argument("--vmesh-study", action="store_true",
                    help="add the uniform-vs-stretched velocity-grid study on the 32^2 cylinder (about 1 minute)")
    ap.add_argument("--refined-study", action="store_true",
                    help="add the refined-vs-uniform velocity-grid study on the Ma-5 cylinder (about 2 minutes)")
    ap.add_argument("--sphere-vmesh-study", action="store_true",
                    help="add the uniform-vs-refined velocity-grid study on the Section 4 sphere (about 10 minutes)")
    ap.add_argument("--slip-study", action="store_true",
                    help="add the wall-slip comparison of the upwind weights, uniform weights and the naive "
                         "extrapolation on the Ma-5 cylinder (about a minute)")
    ap.add_argument("--space-study", action="store_true",
                    help="add the physical-space convergence study of the wall quantities on the cylinder "
                         "(Section 3.3 order estimates; about 5 minutes)")
    ap.add_argument("--cavity-study", action="store_true",
                    help="add the cavity's velocity-space convergence study (about 4 minutes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 512 MiB device copy three times (reference dispatch for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              f"(the step shards by velocity range across GPUs in design, not in code)", file=sys.stderr)
        sys.exit(2)

    from paper_2512_20252_amd import cases

    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    case = cases.cylinder_256(Kn=0.1, Ma=0.3)
    workload = "cylinder_256x256_v48x48"
    tile = tuple(int(x) for x in args.tile.split(",")) if args.tile else None
    tile32 = tuple(int(x) for x in args.tile32.split(",")) if args.tile32 else None
    if args.no_f64:
        r32 = run_gpu(case, "f32", args.steps, args.warmup, tile=tile32)
        print(json.dumps({"f32_ms_per_step": r32["ms"] / args.steps, "tile": r32["tile"], "prof": r32["prof"]}))
        return
    r64 = run_gpu(case, "f64", args.steps, args.warmup, tile=tile)
    upd = r64["nfluid"] * r64["NV"]
    value = upd * args.steps / (r64["ms"] * 1e-3)
    prof = r64["prof"]
    avg_ms = prof["update_ms"] / max(prof["update_launches"], 1)
    bytes_launch = upd * B_ALG[(r64["dim"], "f64")]
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    traffic = _traffic(workload, "f64", r64["tile"])
    ceiling = copy_ceiling()
    line = {
        "metric": "cell*vel updates/s & %HBM peak, FP32-store vs FP64 at fixed C_D err; p50/p99",
        "value": value,
        "unit": "cell*vel updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D cylinder R=0.5 on [-8,8]^2, 256x256 cells, 48x48 velocity nodes on [-6,6]^2, "
                               "Kn 0.1, Ma 0.3, Shakhov, diffuse wall, FP64",
                   "cells": 65536, "fluid_cells": r64["nfluid"], "velocity_nodes": r64["NV"],
                   "timed_as": "one replay of a captured graph of the K steps" if r64["graph"] else "K eager steps"},
        "value_eager": upd * args.steps / (r64["ms_eager"] * 1e-3) if r64["ms_eager"] else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "copy_ceiling_GBs": ceiling["GBs"], "frac_of_copy_ceiling": achieved / ceiling["GBs"],
                     "traffic_GBs": traffic / (avg_ms * 1e-3) / 1e9 if traffic else None,
                     "copy_ceiling": ceiling,
                     "alu": _alu(workload, "f64", r64["tile"], avg_ms),
                     "kernel": "k_update2d<double, %d, %d, false>" % tuple(r64["tile"][:2]),
                     "timing": "HIP events around each update launch on its stream, over K eager steps of this run "
                               "(the steps before the timed graph replay)",
                     "avg_launch_ms": avg_ms, "alg_bytes_per_launch": bytes_launch,
                     "fill_avg_launch_ms": prof["fill_ms"] / max(prof["fill_launches"], 1),
                     "tile": r64["tile"]},
    }
    if not args.no_f32:
        r32 = run_gpu(case, "f32", args.steps, args.warmup, tile=tile32)
        line["precision_form_tile"] = r32["tile"]
        v32 = upd * args.steps / (r32["ms"] * 1e-3)
        avg32 = r32["prof"]["update_ms"] / max(r32["prof"]["update_launches"], 1)
        line["precision_form"] = {"dtype": "f32 storage of f minus the freestream Maxwellian (offsets), "
                                           "f64 moments/equilibrium/wall", "value": v32,
                                  "ratio_vs_f64": v32 / value, "dCD_vs_f64": abs(r32["cd"] - r64["cd"]),
                                  "CD_f64": r64["cd"], "update_avg_launch_ms": avg32,
                                  "update_GBs_alg": upd * 16 / (avg32 * 1e-3) / 1e9,
                                  "update_traffic": _traffic(workload, "f32", r32["tile"]),
                                  "alu": _alu(workload, "f32", r32["tile"], avg32)}
    if args.shard_steps > 0:
        line["shard_shapes"] = shard_shapes(args.shard_steps, args.warmup, value)
    if args.sphere > 0:
        parse = lambda t: tuple(int(x) for x in t.split(",")) if t else None
        line["sphere3d"] = sphere3d(args.sphere, args.sphere_steps, 2,
                                    {"f64": parse(args.sphere_tile), "f32": parse(args.sphere_tile32)})
    if args.hypersonic_steps > 0:
        line["hypersonic"] = hypersonic(args.hypersonic_steps, 2)
    if args.cavity > 0:
        line["cavity"] = cavity(args.cavity, args.cavity_vn, args.cavity_steps, 2, {"f64": None, "f32": None})
    if args.implicit_kn > 0:
        line["implicit_collision"] = implicit_collision(args.implicit_kn, 50, 3)
    if not args.no_fixed_cd:
        fc = fixed_cd_error()
        if fc is not None:
            line["fixed_cd_error"] = fc
            if "precision_form" in line:
                line["precision_form"]["max_dCD_vs_oracle_converged"] = fc["max_dCD_f32_vs_oracle"]
    if args.precision_sweep:
        if args.sweep_sphere_only:
            line["precision_sweep"] = precision_sweep([], 1e-5, 20000)
        else:
            # the cylinder's convergence criterion: C_D moves by less than 1e-6 over 100 steps
            line["precision_sweep"] = precision_sweep(cases.CYLINDER_256_SWEEP, None, 50000, sphere_n=0, atol=1e-6)
    if args.hypersonic_sweep:
        line["precision_sweep_hypersonic"] = precision_sweep([], 1e-6, 30000, sphere_n=0, hypersonic=True)
    if args.vmesh_study:
        line["vmesh_study"] = vmesh_study([8, 12, 16, 24, 32], 128, 30.0, 1.5)
    if args.refined_study:
        line["refined_study"] = refined_study([24, 32, 48], 120, 96, 12.0, 3.0, 1.0,
                                              shapes=[(3.0, 1.0), (2.0, 1.5), (1.0, 1.5)])
    if args.sphere_vmesh_study:
        line["sphere_vmesh_study"] = sphere_vmesh_study(48, [16, 24, 32], 48, 8.0, 2.0, 1.5)
    if args.slip_study:
        line["slip_study"] = slip_study(256, 12.0)
    if args.space_study:
        line["space_study"] = space_study([64, 128, 256], 1024, 0.1, 0.3, 24, 12.0, block=100)
    if args.cavity_study:
        line["cavity_velocity_study"] = cavity_velocity_study(64, [40, 60, 80, 100], 200, 40.0)
    if args.serving > 0:
        line["serving"] = serving(args.serving, args.serving_cap, args.serving_tol, args.serving_gap)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
