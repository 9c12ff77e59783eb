"""Served solves against the oracle directly.  The library draws the
initial perturbation of a served request (and of init_freestream_hashed)
on the device from SplitMix64; the oracle side draws the same published
generator from the seeded-input module (cases.hashed_noise), so both start
from the same state without any value passing from the library to the
oracle.  Bars: FP64 within 1e-12 of the oracle relative to each field's
scale; FP32 storage within 1e-5 relative L2."""
import numpy as np
import pytest

from paper_2512_20252_amd import cases, ibdvm

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
AMP = 1e-3
STEPS = 20

CASES = [cases.cylinder_small(),
         cases.case(dim=2, n=(20, 28), lo=(-1.0, -1.4), hi=(1.0, 1.4), vn=(10, 14), vlo=(-5.0, -5.0),
                    vhi=(5.0, 5.0), geometry="circle", size=(0.35, 0.0, 0.0), Kn=0.05, Ma=1.2, alpha=0.7),
         cases.case(dim=2, n=(24, 24), lo=(-1.2, -1.2), hi=(1.2, 1.2), vn=(16, 16), vlo=(-5.0, -5.0),
                    vhi=(5.0, 5.0), geometry="ellipse", center=(0.0, 0.0, 0.0), size=(0.4, 0.2, 0.0), aoa=0.3,
                    Kn=0.1, Ma=0.8)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _moments_close(mg, mo, tol):
    assert np.array_equal(np.isnan(mg[:, 0]), np.isnan(mo[:, 0]))
    ok = np.isfinite(mo[:, 0])
    for j in (0, 4):
        assert _rel(mg[ok, j], mo[ok, j]) <= tol, j
    T, rho = mo[ok, 4], mo[ok, 0]
    us = max(np.max(np.linalg.norm(mo[ok, 1:4], axis=1)), np.max(np.sqrt(T)))
    qs = max(np.max(np.linalg.norm(mo[ok, 5:8], axis=1)), np.max(rho * T ** 1.5))
    assert np.max(np.abs(mg[ok, 1:4] - mo[ok, 1:4])) <= tol * us
    assert np.max(np.abs(mg[ok, 5:8] - mo[ok, 5:8])) <= tol * qs


def _oracle(oracle_mod, c, seed, steps):
    o = oracle_mod.Oracle(c)
    o.init_freestream(cases.hashed_noise(c, seed), AMP)
    if steps:
        o.step(steps)
    return o


@pytest.mark.parametrize("dim", [2, 3])
def test_hashed_start_matches_oracle(oracle_mod, torch_cuda, dim):
    """The device-drawn start equals f_inf (1 + amp u) with u from the
    published generator, on every cell and node (FP64, to rounding)."""
    c = cases.cylinder_small() if dim == 2 else cases.sphere(n=16, vn=6)
    s = ibdvm.Solver(c, precision="f64")
    s.init_freestream_hashed(77, AMP)
    o = _oracle(oracle_mod, c, 77, 0)
    for a, b in zip(s.get_state(), o.get_state()):
        assert _rel(a, b) <= 4e-16
    s.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("fuse_below", [1 << 62, 0], ids=["fused", "standalone"])
def test_served_solves_match_oracle(oracle_mod, torch_cuda, precision, fuse_below):
    """Three solves of different sizes and physics through one server, all
    in the fused group or all standalone, 20 steps each (two replays of 10),
    against the oracle run from the same seeded start."""
    srv = ibdvm.Server(sum(ibdvm.footprint(c, precision) for c in CASES) + (1 << 20), max_active=3,
                       steps_per_replay=10, fuse_below=fuse_below)
    ids = [srv.submit(c, precision, seed=40 + i, amp=AMP, tol=0.0, max_steps=STEPS, keep_moments=True)
           for i, c in enumerate(CASES)]
    done = {}
    while len(done) < len(ids):
        for r in srv.poll(block=True):
            done[r["id"]] = r
    srv.close()
    for i, (rid, c) in enumerate(zip(ids, CASES)):
        r = done[rid]
        assert r["status"] == ibdvm.OK and r["steps"] == STEPS
        o = _oracle(oracle_mod, c, 40 + i, STEPS)
        mo, mg = o.moments(), r["moments"]
        _, cdo, _, _ = o.forces()
        if precision == "f64":
            _moments_close(mg, mo, TOL64)
            assert abs(r["C_D"] - cdo) <= TOL64 * abs(cdo)
        else:
            ok = np.isfinite(mo[:, 0])
            for j in (0, 1, 2, 4):
                assert np.linalg.norm(mg[ok, j] - mo[ok, j]) / np.linalg.norm(mo[ok, j]) <= 1e-5, j
            assert abs(r["C_D"] - cdo) <= 1e-4


@pytest.mark.parametrize("tile", [(1, 8, 64), (2, 4, 32)])
def test_long_run_unstable_request_steps_match_oracle(oracle_mod, torch_cuda, tile):
    """Request 52 of the 128-request serving stream (a centred 384^2 circle
    at Ma 1.30, Kn 1.9e-3, alpha 0.54, 24^2 nodes), which becomes
    non-physical after about 5000 steps in both storage forms: its first
    steps from the served start agree with the oracle's to 1e-12 (FP64), so
    the library computes the oracle's step on this configuration."""
    reqs, _ = cases.serving_requests(128, 0)
    c = reqs[52]
    o = _oracle(oracle_mod, c, 52, 3)
    s = ibdvm.Solver(c, precision="f64", stream=torch_cuda.cuda.Stream())
    s.set_tile(*tile)
    s.init_freestream_hashed(52, AMP)
    s.step(3)
    _moments_close(s.moments(), o.moments(), TOL64)
    _, cdo, _, _ = o.forces()
    assert abs(s.surface_forces()[1] - cdo) <= TOL64 * abs(cdo)
    s.close()
