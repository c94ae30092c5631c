"""Pins for the oracle's integration set (paper Sec. 5.4) and the claim of Sec. 5.2 that
integrating the closure N loses nothing on the sample particles."""
import copy

import numpy as np
import pytest

import synth
from oracle import closure
from oracle.step import OracleSim


def _brute_force(x, S, n, dx):
    """Sec. 5.4 written out over every grid node: a node is relevant to a position when
    the 1-D quadratic B-spline is non-zero on all three axes (|x / dx - i| < 1.5), and only
    particles whose whole stencil lies inside the grid take part (the build's reading)."""
    def inside(p):
        b = np.floor(x[p] / dx - 0.5)
        return bool(np.all(b >= 0) and np.all(b + 2 <= n - 1))

    def nodes(p):
        out = set()
        for i in range(n):
            if abs(x[p, 0] / dx - i) >= 1.5:
                continue
            for j in range(n):
                if abs(x[p, 1] / dx - j) >= 1.5:
                    continue
                for k in range(n):
                    if abs(x[p, 2] / dx - k) < 1.5:
                        out.add((i, j, k))
        return out

    I = set()
    for s in S:
        if inside(s):
            I |= nodes(s)
    members = [p for p in range(x.shape[0]) if p not in set(S) and inside(p) and nodes(p) & I]
    return list(S) + members


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_closure_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    n, dx = 12, 1.0 / 12
    # some particles near the border, whose stencils leave the grid
    x = rng.uniform(0.02, 0.98, size=(90, 3))
    S = rng.choice(90, size=4, replace=False)
    got = closure.integration_set(x, S, n, dx)
    ref = _brute_force(x, S, n, dx)
    np.testing.assert_array_equal(got, np.asarray(ref))
    # the float32 decision agrees away from ties
    got32 = closure.integration_set_f32(x.astype(np.float32), S, n, np.float32(1.0 / dx))
    np.testing.assert_array_equal(got32, got)


def test_f32_decision_rounds_like_float32():
    """A position whose x / dx - 0.5 is an integer in FP64 but falls just below it in
    float32 arithmetic (or the other way round) takes the float32 base."""
    inv = np.float32(128.0)
    x = np.array([[np.nextafter(np.float32(1.5 / 128), np.float32(0)), 0.5, 0.5]], np.float32)
    b32 = closure.stencil_base_f32(x, inv)
    assert b32[0, 0] == 0
    assert closure.stencil_base_f32(np.array([[1.5 / 128, 0.5, 0.5]], np.float32), inv)[0, 0] == 1


def test_closure_step_loses_nothing_on_the_samples():
    """Sec. 5.2: one MPM step on N gives every sample particle the velocity of the same
    step on all particles (masses V_body / |P| each), to rounding. Dropping a member that
    shares a node with a sample particle changes the result: the pin sees a short N."""
    w = synth.cake_closure(seed=1, r=3, width=16, n=3000, n_sample=6, sigma=0.03,
                           closure_cap=4096, grid_n=32, bias_scale=0.1)
    w.z_prev = w.z0 - 2e-3 * np.random.default_rng(4).normal(size=w.r)
    o = OracleSim(w)
    S = w.plan[0]
    N = o.indices()
    assert 6 < len(N) < 3000
    everyone = np.concatenate([S, np.setdiff1d(np.arange(3000), S)])

    def v_new(idx):
        x, v, tau, C, _ = o.inference(idx)
        return o.mpm_step(x, v, tau, C, len(S))

    v_all = v_new(everyone)
    v_N = v_new(N)
    np.testing.assert_allclose(v_N, v_all, rtol=1e-11, atol=1e-14)
    # a particle of N that shares a node with sample particle 0
    base = closure.stencil_base(o.decode(), w.dx)
    near = [p for p in N[len(S):] if np.all(np.abs(base[p] - base[S[0]]) <= 1)]
    short = N[N != near[0]]
    assert np.abs(v_new(short) - v_all).max() > 1e-9 * np.abs(v_all).max()


def test_closure_trajectory_equals_integrating_everyone():
    """The whole closure-mode step against the plan-mode step whose integration list is
    every particle (S first): same latent trajectory to rounding over 3 steps, with the
    sample set shrunk after the first."""
    w = synth.cake_closure(seed=2, r=3, width=16, n=2000, n_sample=8, sigma=0.03,
                           closure_cap=4096, grid_n=32, bias_scale=0.1)
    w.z_prev = w.z0 - 2e-3 * np.random.default_rng(5).normal(size=w.r)
    a = OracleSim(w)
    w_all = copy.deepcopy(w)
    S = w.plan[0]
    w_all.integration = "plan"
    rest = np.setdiff1d(np.arange(2000), S)
    a.step(1)
    a.set_sample_count(5)
    a.step(2)
    # plan mode: row = S (first 8, then 5) followed by everyone else
    b = OracleSim(w_all)
    w_all.plan = np.concatenate([S, rest])[None, :].astype(np.int32)
    b.step(1)
    w_all.n_sample = 5
    b.n_sample = 5
    w_all.plan = np.concatenate([S[:5], np.setdiff1d(np.arange(2000), S[:5])])[None, :].astype(np.int32)
    b.step(2)
    np.testing.assert_allclose(a.z, b.z, rtol=1e-10, atol=1e-15)
    assert a.flags == b.flags == 0


def test_particle_volume_reading():
    """Closure mode: V_p = V_body / |P| whatever |N|; plan mode: V_body / |N|."""
    w = synth.cake_closure(seed=0, r=3, width=16, n=500, n_sample=4, closure_cap=512, grid_n=32)
    o = OracleSim(w)
    assert o.particle_volume(123) == pytest.approx(w.body_volume / 500)
    w2 = synth.small_cube(seed=0, r=3, width=16, n=256)
    assert OracleSim(w2).particle_volume(256) == pytest.approx(w2.body_volume / 256)
