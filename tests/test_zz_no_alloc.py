"""The network forward that allocates nothing (h4d_mlp_forward_static)
against the ordinary one (h4d_mlp_forward), through the C ABI.

The static entry point reads device features and writes device logits,
keeping the FP32 forward's hidden activations in the library's static
workspace.  Both entry points run the same kernels on the same inputs, so the
logits must agree bit for bit (stronger than the FP32 and BF16 tolerances of
the network's parity tests).  Two calls in a row, the second on fewer rows,
show that the workspace left by a larger call does not leak into a smaller
one.  A size beyond the workspace is refused before any work.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import mlp
from paper_2307_11447_amd import h4d

pytestmark = pytest.mark.gpu


def test_static_forward_equals_forward_on_two_calls():
    import torch
    print("case h4d_mlp_forward_static: 3000 rows then 700, FP32 and BF16", flush=True)
    rng = np.random.default_rng(5)
    net = h4d.Mlp(seed=9)
    net.set_weights(mlp.random_theta(41, scale=1.3))
    L = h4d.lib()
    for bf16 in (False, True):
        for rows in (3000, 700):
            X = (rng.normal(size=(rows, 64)) * 1.5).astype(np.float32)
            ref = net.forward(X, bf16=bf16)
            Xd = torch.from_numpy(X).cuda()
            out = torch.full((rows,), float("nan"), dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            net.forward_static(rows, Xd.data_ptr(), out.data_ptr(), bf16=bf16)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            print(f"   bf16={bf16} rows={rows}: max |diff| {np.abs(got - ref).max():.3e}", flush=True)
            assert np.array_equal(got, ref)
    # beyond the workspace: refused with a message, nothing launched
    big = torch.zeros((4097, 64), dtype=torch.float32, device="cuda")
    out = torch.zeros(4097, dtype=torch.float32, device="cuda")
    rc = L.h4d_mlp_forward_static(net._h, 4097, C.c_void_p(big.data_ptr()), 0, C.c_void_p(out.data_ptr()))
    assert rc == h4d.H4D_EINVAL
    assert b"4096" in L.h4d_last_error()
    rc = L.h4d_mlp_forward_static(net._h, 0, None, 0, None)
    assert rc == h4d.H4D_OK
    net.close()
