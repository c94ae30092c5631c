"""GPU parity of the latent step (HIP path through the C ABI) against the FP64 oracle.

Tolerances (FP32 path). Field values, Jacobians and decoded displacements agree with the
FP64 oracle to FP32 accumulation error: the MLP sums at most 3 + r + 1 and width terms
per layer, so the relative error of an output is a few 1e-7 times a growth factor; 2e-5
of the field's largest magnitude is used. Velocities are backward differences
(u(z_n) - u(z_{n-1})) / dt, so their absolute error is ~2 eps |u| / dt; the G2P velocity
is compared at 1e-3 of its largest magnitude. Trajectories: relative position error
(the paper's delta, Sec. 6) <= 1e-5 after 10 steps at the 1,024-point cube.
"""
import copy

import numpy as np
import pytest
import torch

import synth
from oracle.step import OracleSim, relative_error
from paper_2310_17790_amd import _abi as A
from paper_2310_17790_amd.sim import Sim
from tests.helpers import affine_manifold

pytestmark = pytest.mark.gpu


def _stream():
    return torch.cuda.Stream()


def _soa(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def _with_velocity(w, eps=2e-3, seed=99):
    w = copy.deepcopy(w)
    w.z_prev = w.z0 - eps * np.random.default_rng(seed).normal(size=w.r)
    return w


# (r, width, particles, grid): the ragged and tiny cases, the largest latent (r = 32, split
# over 16 waves per point tile) on the largest grid (256^3: bins of 8^3 cells, 32^3 bins),
# the smallest well-posed sample sets (|S| = r / 3: one particle for r = 3, two for r = 6).
# (6, 128, 8200, 32): enough samples for FP32 team groups of two tiles (257 pairs), the
# last pair with 8 points in its first tile and none in its second
@pytest.mark.parametrize("r,width,n,grid", [(6, 64, 1024, 32), (6, 128, 1000, 32), (24, 128, 515, 32),
                                            (1, 64, 77, 32), (3, 64, 96, 32), (32, 128, 700, 256),
                                            (3, 64, 1, 32), (6, 64, 2, 32), (6, 128, 8200, 32)])
def test_stage_parity_one_step(r, width, n, grid):
    w = _with_velocity(synth.small_cube(seed=3, r=r, width=width, n=n, bias_scale=0.1))
    w.grid_n, w.dx = grid, 1.0 / grid
    print(f"\n[case] stage parity r={r} width={width} n={n} grid={grid}", flush=True)
    s = _stream()
    sim = Sim(w, stream=s)
    # the field inference of step 0 (and the decode at z0), as the step will consume it
    sim.refresh(stream=s)
    s.synchronize()
    o = OracleSim(w)
    x0 = _soa(sim.buffer(A.NSF_BUF_XDEC)).reshape(3, -1).T
    errs0 = _rel_max(x0 - o.X, o.decode() - o.X)
    idx = o.indices(0)
    x, v, tau, C, u_n = o.inference(idx)
    XN = o.X[idx]
    u_prev = o.u(XN, o.z_prev)
    N, S = w.n_integration, w.n_sample
    errs = {}
    errs["u"] = _rel_max(_soa(sim.buffer(A.NSF_BUF_U)).reshape(3, N).T, u_n)
    errs["u_prev"] = _rel_max(_soa(sim.buffer(A.NSF_BUF_UPREV)).reshape(3, N).T, u_prev)
    t6 = _soa(sim.buffer(A.NSF_BUF_TAU)).reshape(6, N).T
    voigt = np.stack([tau[:, 0, 0], tau[:, 1, 1], tau[:, 2, 2], tau[:, 1, 2], tau[:, 0, 2], tau[:, 0, 1]], 1)
    errs["tau"] = _rel_max(t6, voigt)
    errs["C"] = _rel_max(_soa(sim.buffer(A.NSF_BUF_C)).reshape(9, N).T, C.reshape(N, 9))
    J = o.jac(XN[:S], o.z)                              # (S, 3, r)
    Jg = _soa(sim.buffer(A.NSF_BUF_JAC)).reshape(3, r, S).transpose(2, 0, 1)
    errs["J"] = _rel_max(Jg, J)
    errs["decode_u"] = errs0
    u_gpu = _soa(sim.buffer(A.NSF_BUF_U)).reshape(3, N).T
    sim.step(1, stream=s)
    s.synchronize()
    v_new = o.mpm_step(x, v, tau, C, S)
    errs["v_new"] = _rel_max(_soa(sim.buffer(A.NSF_BUF_VNEW)).reshape(3, S).T, v_new)
    z_ref = o.inversion(XN[:S], u_n[:S] + w.dt * v_new)
    z_gpu, zp_gpu, st = sim.latent()
    # the latent's error is the velocity's (FP32 backward difference) carried through the
    # Gauss-Newton step, so it is measured against the step z_{n+1} - z_n
    errs["dz"] = float(np.abs(z_gpu - z_ref).max() / np.abs(z_ref - w.z0).max())
    # Gauss-Newton parity on its own: the oracle's inversion fed the GPU's G2P velocity.
    # (With r = 24 the normal equations are ill-conditioned enough that the velocity's
    # FP32 error, not the solver, dominates dz.)
    v_gpu = _soa(sim.buffer(A.NSF_BUF_VNEW)).reshape(3, S).T
    z_ref2 = o.inversion(XN[:S], u_n[:S] + w.dt * v_gpu)
    errs["gn"] = float(np.abs(z_gpu - z_ref2).max() / np.abs(z_ref2 - w.z0).max())
    Jm = J.reshape(-1, r)
    errs["cond_J"] = float(np.linalg.cond(Jm))
    print("errors:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert st == 1
    np.testing.assert_array_equal(zp_gpu, w.z0)
    for k in ("u", "u_prev", "tau", "C", "J"):
        assert errs[k] < 2e-5, (k, errs[k])
    # decoded positions x = X + u are FP32 values near |X| ~ 0.5: their rounding (half an
    # ulp of x) adds up to 2^-24 max|x| / max|u| to the relative displacement error
    u_ref = o.decode() - o.X
    tol_dec = 2e-5 + 2.0 ** -24 * np.abs(o.X).max() / np.abs(u_ref).max()
    assert errs["decode_u"] < tol_dec, (errs["decode_u"], tol_dec)
    # velocities are (u(z_n) - u(z_{n-1})) / dt of FP32 field values: absolute error ~ 2 eps_u / dt
    v_gpu = _soa(sim.buffer(A.NSF_BUF_VNEW)).reshape(3, S).T
    eps_u = float(np.abs(u_gpu - u_n).max())
    tol_v = 1e-4 + 10 * eps_u / (w.dt * np.abs(v_new).max())
    assert errs["v_new"] < tol_v, (errs["v_new"], tol_v)
    # The second iterate's residual subtracts two FP32 field values, so each of its 3 S
    # entries carries an absolute error of up to ~2 eps_u; to first order the least-squares
    # solution then moves by at most |dr|_2 / sigma_min(J), and the Jacobian's own relative
    # error e_J moves it by up to cond(J) e_J relative. Both are taken with a factor 10.
    du_step = float(w.dt * np.abs(v_gpu).max())
    sig_min = float(np.linalg.svd(Jm, compute_uv=False)[-1])
    dz_ref = float(np.abs(z_ref2 - w.z0).max())
    tol_gn = 1e-4 + 10 * (2 * np.sqrt(3 * S) * eps_u / sig_min) / dz_ref + 10 * errs["cond_J"] * errs["J"]
    print(f"tol_gn={tol_gn:.2e} (eps_u={eps_u:.2e}, sigma_min={sig_min:.2e}, |dz|={dz_ref:.2e}, "
          f"dt|v|={du_step:.2e})", flush=True)
    assert errs["gn"] < tol_gn
    # end to end: the velocity's relative error (<= 1e-3) amplified by at most cond(J)
    assert errs["dz"] < tol_gn + 1e-3 * max(1.0, errs["cond_J"] / 10)
    assert sim.flags() == (0, 0)
    # P2G + grid update: node mass and new velocity where the oracle has mass
    from oracle import mpm
    nN = x.shape[0]
    V = np.full(nN, w.body_volume / nN)
    Am = mpm.affine_matrix(C, tau, w.rho * V, V, w.dt, w.dx)
    mass, mom, _ = mpm.p2g(x, v, Am, w.rho * V, w.grid_n, w.dx)
    vel = mpm.grid_update(mass, mom, w.grid_n, w.dx, w.dt, w.gravity, w.wall_nodes, w.dt, w.knife)
    grid = _soa(sim.buffer(A.NSF_BUF_GRID)).reshape(-1, 4)
    has = mass > 0
    assert _rel_max(grid[has, 3], mass[has]) < 1e-5
    assert _rel_max(grid[has, :3], vel[has]) < tol_v


def test_cube_trajectory_10_steps():
    """The 1,024-point cube: 10 steps, 2 Gauss-Newton iterations, FP32 GPU vs FP64."""
    w = _with_velocity(synth.small_cube(seed=0, r=6, width=64, n=1024, steps=10))
    print("\n[case] cube trajectory 10 steps", flush=True)
    s = _stream()
    sim = Sim(w, stream=s)
    o = OracleSim(w)
    worst = 0.0
    for k in range(10):
        sim.step(1, stream=s)
        o.step(1)
        s.synchronize()
        xg = _soa(sim.buffer(A.NSF_BUF_XDEC)).reshape(3, -1).T
        xo = o.decode()
        d = relative_error(xg, xo)
        du = relative_error(xg - o.X, xo - o.X)
        zg, _, _ = sim.latent()
        print(f"step {k + 1}: delta_x={d:.2e} delta_u={du:.2e} dz={np.abs(zg - o.z).max():.2e}", flush=True)
        worst = max(worst, d)
    assert worst <= 1e-5
    assert sim.flags() == (0, 0)


def test_slab_sampled_knife_ragged():
    """Width 128, 3,000 particles, 1,000 integration (ragged tile) of which 700 sample,
    knife on, 64^3 grid, 3 steps."""
    w = synth.cake_slab(seed=5, r=6, width=128, n=3000, n_integration=1000, steps=3,
                        grid_n=64, bias_scale=0.05)
    w.n_sample = 700
    w.knife.edge_z0 = 0.1
    w = _with_velocity(w)
    print("\n[case] slab sampled knife ragged", flush=True)
    s = _stream()
    sim = Sim(w, stream=s)
    o = OracleSim(w)
    for k in range(3):
        sim.step(1, stream=s)
        o.step(1)
        s.synchronize()
        xg = _soa(sim.buffer(A.NSF_BUF_XDEC)).reshape(3, -1).T
        d = relative_error(xg, o.decode())
        zg, _, _ = sim.latent()
        print(f"step {k + 1}: delta_x={d:.2e} dz={np.abs(zg - o.z).max():.2e}", flush=True)
        assert d <= 1e-5
    assert sim.flags() == (0, 0)


def test_affine_manifold_free_fall_on_gpu():
    w = affine_manifold(synth.small_cube(seed=0, r=3, width=64, n=256))
    print("\n[case] affine free fall", flush=True)
    s = _stream()
    sim = Sim(w, stream=s)
    x0 = _soa(sim.decode(stream=s)).T
    n = 6
    sim.step(n, stream=s)
    s.synchronize()
    xg = _soa(sim.buffer(A.NSF_BUF_XDEC)).reshape(3, -1).T
    expect = x0 + np.asarray(w.gravity)[None, :] * w.dt ** 2 * n * (n + 1) / 2
    err = np.abs(xg - expect).max()
    print(f"free fall max err {err:.2e} (displacement {abs(w.gravity[2]) * w.dt ** 2 * n * (n + 1) / 2:.2e})")
    assert err < 2e-7


def test_decode_user_points_ragged():
    w = synth.small_cube(seed=4, r=6, width=128, n=256, bias_scale=0.1)
    print("\n[case] decode user points", flush=True)
    s = _stream()
    sim = Sim(w, stream=s)
    Xq = synth.box_points(77, 77, (0.3, 0.3, 0.3), (0.7, 0.7, 0.7))
    out = sim.decode(torch.from_numpy(Xq).cuda(), stream=s)
    s.synchronize()
    o = OracleSim(w)
    ref = o.decode(Xq.T.astype(np.float64))
    du = _rel_max(_soa(out).T - Xq.T, ref - Xq.T)
    print(f"decode du rel {du:.2e}")
    assert du < 2e-5


def test_resume_from_latent_checkpoint():
    w = _with_velocity(synth.small_cube(seed=6, r=6, width=64, n=512, steps=4))
    s = _stream()
    a = Sim(w, stream=s)
    a.step(4, stream=s)
    za, zpa, sta = a.latent(stream=s)
    b = Sim(w, stream=s)
    b.step(2, stream=s)
    z, zp, st = b.latent(stream=s)
    c = Sim(w, stream=s)
    c.set_latent(z, zp, st, stream=s)
    c.step(2, stream=s)
    zc, zpc, stc = c.latent(stream=s)
    assert sta == stc == 4
    # the step is deterministic: resuming from the checkpoint gives the same bits
    np.testing.assert_array_equal(zc, za)
    np.testing.assert_array_equal(zpc, zpa)
    # and both match the oracle's 4-step latent to the trajectory tolerance
    o = OracleSim(w)
    o.step(4)
    motion = np.abs(o.z - w.z0).max()
    for zz in (za, zc):
        assert np.abs(zz - o.z).max() <= 1e-3 * motion + 1e-7


def test_flags_nonfinite_and_domain():
    w = synth.small_cube(seed=7, r=6, width=64, n=256)
    s = _stream()
    sim = Sim(w, stream=s)
    z = np.array(w.z0)
    z[0] = np.nan
    sim.set_latent(z, stream=s)
    sim.step(1, stream=s)
    st, f = sim.flags(stream=s)
    assert f & A.NSF_FLAG_NONFINITE
    assert st == A.NSF_ENONFINITE
    # a point outside the grid: shift every reference position to the domain edge
    w2 = copy.deepcopy(w)
    w2.X = w2.X.copy()
    w2.X[0, 0] = 0.001
    sim2 = Sim(w2, stream=s)
    sim2.step(1, stream=s)
    st2, f2 = sim2.flags(stream=s)
    assert f2 & A.NSF_FLAG_DOMAIN and st2 == A.NSF_EDOMAIN
    o = OracleSim(w2)
    o.step(1)
    assert o.flags & o.FLAG_DOMAIN


@pytest.mark.parametrize("precision,gn_iters,damping", [("fp32", 1, 0.0), ("fp32", 3, 0.0), ("fp32", 2, 0.05),
                                                        ("fp32", 3, 0.5), ("bf16", 2, 0.05)])
def test_inversion_variants(precision, gn_iters, damping):
    """The first-order projection (one solve with J(z_n)), three iterations, and
    Levenberg-Marquardt damping: 5 steps of the cube against the oracle run with the same
    settings (FP32 gate 1e-5, BF16 gate 1e-4 on delta_x). Where a setting moves the latent
    well beyond the GPU's rounding (all but three undamped iterations, which agree with
    two to ~3e-6), the GPU latent must sit far closer to the oracle with that setting
    than to the default two undamped iterations: the option reaches the kernels."""
    w = _with_velocity(synth.small_cube(seed=0, r=6, width=64, n=1024, steps=5))
    w.gn_iters, w.gn_damping = gn_iters, damping
    print(f"\n[case] inversion variant {precision} gn_iters={gn_iters} damping={damping}", flush=True)
    s = _stream()
    sim = Sim(w, precision=precision, stream=s)
    o = OracleSim(w)
    gate = 1e-5 if precision == "fp32" else 1e-4
    for k in range(5):
        sim.step(1, stream=s)
        o.step(1)
        s.synchronize()
        xg = _soa(sim.buffer(A.NSF_BUF_XDEC)).reshape(3, -1).T
        d = relative_error(xg, o.decode())
        zg, _, st = sim.latent(stream=s)
        print(f"step {k + 1}: delta_x={d:.2e} dz={np.abs(zg - o.z).max():.2e}", flush=True)
        assert st == k + 1
        assert d <= gate
    assert sim.flags(stream=s) == (0, 0)
    base = copy.deepcopy(w)
    base.gn_iters, base.gn_damping = 2, 0.0
    ob = OracleSim(base)
    ob.step(5)
    apart = float(np.abs(o.z - ob.z).max())
    err = float(np.abs(zg - o.z).max())
    print(f"|z_variant - z_default| = {apart:.2e}, |z_gpu - z_variant| = {err:.2e}", flush=True)
    if not (gn_iters == 3 and damping == 0.0):
        assert err < 0.1 * apart
    sim.close()


def test_problem_parameters_on_gpu():
    """h(X, z, mu) with two parameters: the stress of the inference against the oracle's
    (FP32 gate 2e-5), again after nsf_set_parameters, and 4 steps with the parameter
    changed after the second (delta_x <= 1e-5). The change must move the stress far more
    than the FP32 error (the parameters reach the kernel)."""
    w = _with_velocity(synth.small_cube(seed=6, r=6, width=128, n=1000, steps=4, bias_scale=0.1))
    w.fields = synth.make_fields(6, 6, 128, bias_scale=0.1, n_mu=2)
    w.mu = np.array([0.4, -0.8])
    print("\n[case] problem parameters n_mu=2 width=128", flush=True)
    s = _stream()
    sim = Sim(w, stream=s)
    o = OracleSim(w)
    N = w.n_integration

    def tau_err():
        sim.refresh(stream=s)
        s.synchronize()
        _, _, tau, _, _ = o.inference(o.indices())
        t6 = _soa(sim.buffer(A.NSF_BUF_TAU)).reshape(6, N).T
        voigt = np.stack([tau[:, 0, 0], tau[:, 1, 1], tau[:, 2, 2], tau[:, 1, 2], tau[:, 0, 2], tau[:, 0, 1]], 1)
        return _rel_max(t6, voigt), t6

    e0, t_a = tau_err()
    sim.set_parameters([-0.3, 1.1], stream=s)
    o.set_parameters([-0.3, 1.1])
    e1, t_b = tau_err()
    moved = float(np.abs(t_b - t_a).max() / np.abs(t_a).max())
    print(f"tau errors {e0:.2e} {e1:.2e}; change with mu {moved:.2e}", flush=True)
    assert e0 < 2e-5 and e1 < 2e-5 and moved > 1e-3
    for k in range(4):
        if k == 2:
            sim.set_parameters([0.9, 0.0], stream=s)
            o.set_parameters([0.9, 0.0])
        sim.step(1, stream=s)
        o.step(1)
        s.synchronize()
        d = relative_error(_soa(sim.buffer(A.NSF_BUF_XDEC)).reshape(3, -1).T, o.decode())
        print(f"step {k + 1}: delta_x={d:.2e}", flush=True)
        assert d <= 1e-5
    assert sim.flags(stream=s) == (0, 0)
    with pytest.raises(A.NsfError):
        sim.set_parameters([1.0], stream=s)
    sim.close()
