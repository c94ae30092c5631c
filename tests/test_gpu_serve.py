"""The continuous-batching server on the GPU: requests that arrive while others run are
admitted as memory frees up, their steps share launches, and every request's result is
bit for bit the one it gets alone (the step is deterministic and sims share no state)."""
import numpy as np
import pytest
import torch

import synth
from paper_2310_17790_amd.serve import GpuBackend, Request, Server
from paper_2310_17790_amd.sim import Sim

pytestmark = pytest.mark.gpu


def _requests():
    specs = [(6000, 6, 64, 60), (3000, 12, 32, 40), (9000, 6, 64, 50), (4000, 12, 64, 30),
             (7000, 6, 32, 45), (5000, 12, 64, 35)]
    out = []
    for i, (n, r, g, steps) in enumerate(specs):
        req = dict(n_particles=n, n_integration=int(0.08 * n), r=r, grid_n=g, weight_seed=2000 + i)
        w = synth.served_instance(req, width=128, steps=steps, plan_steps=4)
        w.z_prev = w.z0 - 1e-3 * np.random.default_rng(i).normal(size=r)
        out.append(Request(i, arrival_s=0.001 * i, workload=w, steps=steps, keep_positions=True))
    return out


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_served_mix_equals_solo(precision):
    print(f"\n[case] served mix {precision}", flush=True)
    reqs = _requests()
    be = GpuBackend(precision=precision)
    budget = 3 * max(Sim.bytes_for(q.workload, precision) for q in reqs)
    srv = Server(be, hbm_budget_bytes=budget)
    srv.submit(reqs)
    st = srv.run()
    print({k: st[k] for k in ("requests", "ticks", "peak_active", "p50_step_ms", "p99_step_ms")}, flush=True)
    assert st["requests"] == len(reqs) and st["failed"] == 0
    assert st["peak_active"] >= 2 and srv.peak_used <= budget
    s = torch.cuda.Stream()
    for res in srv.results:
        q = reqs[res.rid]
        solo = Sim(q.workload, precision=precision, stream=s)
        solo.step(q.steps, stream=s)
        z, _, step = solo.latent(stream=s)
        assert step == q.steps
        np.testing.assert_array_equal(res.z, z)
        x = solo.buffer(5 + 1).reshape(3, -1).cpu().numpy()   # NSF_BUF_XDEC
        np.testing.assert_array_equal(res.positions, x)
        solo.close()
