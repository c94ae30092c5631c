"""The allocation-free field forward (nsf_mlp_forward_noalloc) against nsf_mlp_forward.

Both run the same packing and field kernels, the first with its packed weights in the
library's per-device array, the second in a caller workspace, so outputs and saved
pre-activations must agree bit for bit. Two calls in a row, the second smaller (fewer
points, a smaller latent, another width and output count), show that the array is
reused and that nothing of the first call's packing leaks into the second.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from paper_2310_17790_amd import _abi as A
from paper_2310_17790_amd.sim import flatten_mlp

pytestmark = pytest.mark.gpu


def _case(seed, r, width, d, n):
    w = synth.small_cube(seed=seed, r=r, width=width, n=64, steps=1)
    name = {3: "g", 6: "h", 9: "l"}[d]
    weights = torch.from_numpy(flatten_mlp(w.fields[name])).cuda()
    g = np.random.default_rng(seed + 7)
    X = torch.from_numpy(g.uniform(0.3, 0.7, size=(3, n)).astype(np.float32)).cuda()
    Z = torch.from_numpy(g.normal(0.0, 0.3, size=(n, r)).astype(np.float32)).cuda()
    return weights, X, Z


def _mlp(weights, r, width, d, precision):
    m = A.nsf_mlp()
    m.r, m.width, m.d = r, width, d
    m.precision = A.NSF_BF16 if precision == "bf16" else A.NSF_FP32
    m.weights = weights.data_ptr()
    return m


def _forward(L, m, X, Z, n, width, d, noalloc, stream):
    out = torch.full((d, n), float("nan"), dtype=torch.float32, device="cuda")
    saved = torch.full((L.nsf_mlp_saved_floats(width, n),), float("nan"), dtype=torch.float32,
                       device="cuda")
    if noalloc:
        st = L.nsf_mlp_forward_noalloc(C.byref(m), X.data_ptr(), Z.data_ptr(), n, out.data_ptr(),
                                       saved.data_ptr(), stream)
    else:
        nb = L.nsf_mlp_workspace_bytes(C.byref(m), n)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        st = L.nsf_mlp_forward(C.byref(m), X.data_ptr(), Z.data_ptr(), n, out.data_ptr(),
                               saved.data_ptr(), ws.data_ptr(), nb, stream)
    A.check(st)
    torch.cuda.synchronize()
    return out.cpu(), saved.cpu()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_forward_matches_workspace_forward(precision):
    L = A.lib()
    stream = int(torch.cuda.current_stream().cuda_stream)
    # the largest shape first, then a smaller one on the same array
    for seed, r, width, d, n in [(3, 32, 128, 9, 5003), (4, 6, 64, 3, 517)]:
        print(f"noalloc {precision}: r={r} width={width} d={d} n={n}", flush=True)
        weights, X, Z = _case(seed, r, width, d, n)
        m = _mlp(weights, r, width, d, precision)
        ref_out, ref_saved = _forward(L, m, X, Z, n, width, d, False, stream)
        out, saved = _forward(L, m, X, Z, n, width, d, True, stream)
        assert torch.isfinite(ref_out).all()
        assert torch.equal(out, ref_out)
        # bit patterns: BF16 training fills the first half of the buffer and leaves the
        # rest (NaN here) as it was
        assert torch.equal(saved.view(torch.int32), ref_saved.view(torch.int32))


def test_noalloc_forward_rejects_invalid_arguments():
    L = A.lib()
    stream = int(torch.cuda.current_stream().cuda_stream)
    weights, X, Z = _case(5, 6, 64, 3, 32)
    out = torch.empty((3, 32), dtype=torch.float32, device="cuda")
    m = _mlp(weights, 6, 64, 3, "fp32")
    assert L.nsf_mlp_forward_noalloc(C.byref(m), X.data_ptr(), Z.data_ptr(), 32, None, None,
                                     stream) == A.NSF_EINVAL
    m.width = 96
    assert L.nsf_mlp_forward_noalloc(C.byref(m), X.data_ptr(), Z.data_ptr(), 32, out.data_ptr(),
                                     None, stream) == A.NSF_EINVAL
