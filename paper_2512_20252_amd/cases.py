"""Workload descriptions and seeded synthetic inputs.

This module holds parameter values and random draws only; none of the
method's arithmetic lives here, so the HIP library and the CPU oracle can
both consume its outputs without sharing any computation.

A case is a plain dict: grid (dim, n, lo, hi, outer), velocity grid (vn, vlo,
vhi, rule), geometry (geometry, center, size, aoa), physics (Kn, Ma, Pr,
gamma, alpha, Tw) and numerics (cfl, omega_vhs, a_vhs, flags).
"""
import numpy as np

BASE = dict(Pr=2.0 / 3.0, gamma=5.0 / 3.0, alpha=1.0, Tw=1.0, cfl=0.5, omega_vhs=0.81, a_vhs=1.0,
            outer="freestream", rule="midpoint", geometry="none", center=(0.0, 0.0, 0.0),
            size=(0.0, 0.0, 0.0), aoa=0.0, flags=(), lid_u=0.0)


def case(**kw):
    c = dict(BASE)
    c.update(kw)
    return c


def cylinder_small():
    """2D cylinder, plain FP64: [-1,1]^2 on 32x32, R=0.3, 16x16 trapezoid
    velocity grid on [-5,5]^2, Ma 0.5, Kn 0.1, diffuse wall at T_inf."""
    return case(dim=2, n=(32, 32), lo=(-1.0, -1.0), hi=(1.0, 1.0), vn=(16, 16), vlo=(-5.0, -5.0),
                vhi=(5.0, 5.0), rule="trapezoid", geometry="circle", size=(0.3, 0.0, 0.0),
                Kn=0.1, Ma=0.5)


def cylinder_256(Kn=0.1, Ma=0.3, n=256, vn=48):
    """2D cylinder: [-8,8]^2 on 256x256, R=0.5, 48x48 midpoint velocity grid
    on [-6,6]^2 (the throughput workload)."""
    return case(dim=2, n=(n, n), lo=(-8.0, -8.0), hi=(8.0, 8.0), vn=(vn, vn), vlo=(-6.0, -6.0),
                vhi=(6.0, 6.0), geometry="circle", size=(0.5, 0.0, 0.0), Kn=Kn, Ma=Ma)


def cylinder_256_velocity_shard(G=8, Kn=0.1, Ma=0.3, n=256, vn=48):
    """The per-GPU shape of the 256^2 cylinder when its vn x vn velocity grid
    is split over G GPUs by interleaved rows (GPU g owning the nodes whose y
    index is g modulo G): the same cells with a vn x (vn/G) midpoint grid on
    the same box [-6,6]^2, whose y spacing is G times the full grid's like
    that of a share.  A share's own nodes are offset from these by a
    fraction of a spacing (the library takes velocity boxes symmetric about
    0 only); the update does the same work for any node values.  Run alone
    it is a coarse velocity grid of the same flow."""
    if vn % G:
        raise ValueError("the shard count must divide the nodes per axis")
    return case(dim=2, n=(n, n), lo=(-8.0, -8.0), hi=(8.0, 8.0), vn=(vn, vn // G), vlo=(-6.0, -6.0),
                vhi=(6.0, 6.0), geometry="circle", size=(0.5, 0.0, 0.0), Kn=Kn, Ma=Ma)


def cylinder_256_slab(G=8, Kn=0.1, Ma=0.3, n=256, vn=48):
    """The per-GPU shape of the 256^2 cylinder split over G GPUs into slabs
    of n/G rows, for the slab that carries the body: n x n/G cells of the
    same spacing centred on the cylinder ([-8,8] x [-8/G,8/G]), the full
    vn x vn velocity grid, freestream rows beyond the slab where a share
    would read its neighbours' halo rows."""
    if n % G:
        raise ValueError("the slab count must divide the rows")
    h = 8.0 / G
    return case(dim=2, n=(n, n // G), lo=(-8.0, -h), hi=(8.0, h), vn=(vn, vn), vlo=(-6.0, -6.0),
                vhi=(6.0, 6.0), geometry="circle", size=(0.5, 0.0, 0.0), Kn=Kn, Ma=Ma)


CYLINDER_256_SWEEP = [(Kn, Ma) for Kn in (0.01, 0.1, 1.0) for Ma in (0.3, 2.0)]


def hypersonic_bodies(seed=0, nx=512, ny=384, vn=64):
    """2D ellipse and symmetric 4-digit airfoil at Ma 5, Kn 0.05, alpha 0.8 on
    [-3,7]x[-3.75,3.75]; thickness t~U(0.08,0.2), angle of attack ~U(0,8 deg)
    and ellipse aspect ~U(1,4) drawn in that order from the seed."""
    rng = np.random.default_rng(seed)
    t = float(rng.uniform(0.08, 0.2))
    aoa = float(np.deg2rad(rng.uniform(0.0, 8.0)))
    aspect = float(rng.uniform(1.0, 4.0))
    common = dict(dim=2, n=(nx, ny), lo=(-3.0, -3.75), hi=(7.0, 3.75), vn=(vn, vn), vlo=(-10.0, -10.0),
                  vhi=(10.0, 10.0), Kn=0.05, Ma=5.0, alpha=0.8)
    airfoil = case(geometry="airfoil", center=(0.0, 0.0, 0.0), size=(1.0, t, 0.0), aoa=aoa, **common)
    ellipse = case(geometry="ellipse", center=(0.5, 0.0, 0.0), size=(0.5, 0.5 / aspect, 0.0), aoa=aoa, **common)
    return airfoil, ellipse


def sphere(n=96, vn=24):
    """3D sphere R=0.5 in [-4,4]^3, full distribution on a vn^3 midpoint grid
    on [-6,6]^3, Kn 0.1, Ma 1.5, diffuse wall at T_inf."""
    return case(dim=3, n=(n, n, n), lo=(-4.0, -4.0, -4.0), hi=(4.0, 4.0, 4.0), vn=(vn, vn, vn),
                vlo=(-6.0, -6.0, -6.0), vhi=(6.0, 6.0, 6.0), geometry="sphere", size=(0.5, 0.0, 0.0),
                Kn=0.1, Ma=1.5)


def cavity(n=64, vn=40, Kn=0.075, lid_u=0.15):
    """Lid-driven cavity with a stationary cylinder (Section 4 convergence
    test): unit square, n^2 cells, diffuse walls at T_w = 1 with the top wall
    moving at lid_u along x, cylinder of diameter 0.25 at the centre,
    vn^2 midpoint velocity grid on [-5,5]^2, gas initially at rest."""
    return case(dim=2, n=(n, n), lo=(0.0, 0.0), hi=(1.0, 1.0), outer="walls", lid_u=lid_u, vn=(vn, vn),
                vlo=(-5.0, -5.0), vhi=(5.0, 5.0), geometry="circle", center=(0.5, 0.5, 0.0),
                size=(0.125, 0.0, 0.0), Kn=Kn, Ma=0.0)


def n_cells(c):
    return int(np.prod(c["n"][: c["dim"]]))


def n_vel(c):
    return int(np.prod(c["vn"][: c["dim"]]))


def noise(c, seed=0):
    """Uniform(-1,1) perturbation fields, one per distribution array (h then b
    in 2D; f in 3D), each of shape (cells, velocity nodes) in C order, drawn
    from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    shape = (n_cells(c), n_vel(c))
    na = 2 if c["dim"] == 2 else 1
    return tuple(rng.uniform(-1.0, 1.0, size=shape) for _ in range(na))


def splitmix64_uniform(seed, start, count):
    """Uniform values in [-1, 1) from SplitMix64 (Steele, Lea and Flood,
    OOPSLA 2014): output j of the generator seeded with `seed` is the
    finaliser applied to seed + j * 0x9e3779b97f4a7c15, j = start + 1 ...
    start + count; the top 53 bits, scaled by 2^-52, minus 1.  The library
    draws the perturbation of its device-side initial state (and of served
    requests) from the same published generator, with j - 1 running over
    (array, cell, node) in storage order."""
    z = np.uint64(seed) + (np.arange(start, start + count, dtype=np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


def hashed_noise(c, seed):
    """The perturbation fields of a seeded device-side start (one per
    distribution array, shape (cells, velocity nodes)): SplitMix64 values
    with the array index running first, then cell, then node."""
    n = n_cells(c) * n_vel(c)
    na = 2 if c["dim"] == 2 else 1
    return tuple(splitmix64_uniform(seed, A * n, n).reshape(n_cells(c), n_vel(c)) for A in range(na))


def serving_requests(n=128, seed=0):
    """Seeded stream of 2D solve requests of mixed sizes on [-4,4]^2: grid
    N in {64, 96, ..., 384}, velocity grid N_xi in {16, 24, ..., 56} on
    [-V, V]^2 with V = max(6, ceil(U_inf + 4 sqrt(1 + Ma^2/3))), geometry
    uniform over cylinder (r ~ U(0.2, 0.6)), ellipse (chord 1, aspect ~
    U(1, 4)) and airfoil (chord 1, t ~ U(0.08, 0.2)), Kn log-uniform on
    [1e-3, 1], Ma ~ U(0.2, 3), alpha ~ U(0.5, 1).  Fields are drawn per
    request in that order, then the arrival gaps as unit-mean exponentials
    (scaled by the caller)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        N = int(rng.choice(np.arange(64, 385, 32)))
        nxi = int(rng.choice(np.arange(16, 57, 8)))
        kind = int(rng.integers(0, 3))
        shape = float(rng.uniform(0.2, 0.6)) if kind == 0 else (float(rng.uniform(1.0, 4.0)) if kind == 1
                                                                else float(rng.uniform(0.08, 0.2)))
        Kn = float(10.0 ** rng.uniform(-3.0, 0.0))
        Ma = float(rng.uniform(0.2, 3.0))
        alpha = float(rng.uniform(0.5, 1.0))
        U = Ma * np.sqrt(5.0 / 6.0)
        V = float(max(6.0, np.ceil(U + 4.0 * np.sqrt(1.0 + Ma * Ma / 3.0))))
        common = dict(dim=2, n=(N, N), lo=(-4.0, -4.0), hi=(4.0, 4.0), vn=(nxi, nxi), vlo=(-V, -V), vhi=(V, V),
                      Kn=Kn, Ma=Ma, alpha=alpha)
        if kind == 0:
            c = case(geometry="circle", size=(shape, 0.0, 0.0), **common)
        elif kind == 1:
            c = case(geometry="ellipse", center=(0.0, 0.0, 0.0), size=(0.5, 0.5 / shape, 0.0), **common)
        else:
            c = case(geometry="airfoil", center=(-0.5, 0.0, 0.0), size=(1.0, shape, 0.0), **common)
        out.append(c)
    gaps = rng.exponential(1.0, size=n)
    return out, gaps
