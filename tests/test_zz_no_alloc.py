"""The allocation-free gradient entry point (jg_mlp_grad_noalloc) against jg_mlp_grad, through
the C ABI: two calls in a row, the second with a smaller batch.  Both run the same kernels with
the same launch shape, so gradient and loss agree bit for bit."""
import sys

import numpy as np
import pytest

from oracle import mlp as M
from paper_2606_28394_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _params(seed):
    flat = W.mlp_init(seed)
    P = M.unpack(flat)
    rng = np.random.default_rng(300 + seed)
    P["mean"][:] = rng.normal(0.0, 0.5, 24)
    P["std"][:] = rng.uniform(0.5, 2.0, 24)
    return flat.astype(np.float32)


def test_noalloc_gradient_matches_workspace_gradient():
    import torch
    from paper_2606_28394_amd import jenga as J
    fn = J.load_library().jg_mlp_grad_noalloc
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    net = J.Mlp(_params(5))
    for n in (40_000, 777):
        _say(f"no-alloc gradient: batch {n}")
        rng = np.random.default_rng(n)
        F = torch.as_tensor(W.random_features(n, 7 + n).astype(np.float32)).cuda()
        T = torch.as_tensor(rng.normal(0.0, 0.3, (n, 3)).astype(np.float32)).cuda()
        g_ref, l_ref = net.compute_grad(F, T)
        g_ref, l_ref = g_ref.clone(), l_ref.clone()
        g = torch.full((J.MLP_TRAINABLE,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        rc = fn(net.params.data_ptr(), net.packed.data_ptr(), F.data_ptr(), T.data_ptr(), n, g.data_ptr(),
                loss.data_ptr(), stream)
        assert rc == J.JG_OK, J.jg_last_error()
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), float((g - g_ref).abs().max())
        assert torch.equal(loss, l_ref)
        assert torch.isfinite(g).all() and float(g.abs().max()) > 0.0
    # an empty batch is refused before any launch
    assert fn(net.params.data_ptr(), net.packed.data_ptr(), F.data_ptr(), T.data_ptr(), 0, g.data_ptr(),
              loss.data_ptr(), stream) == J.JG_EINVAL
