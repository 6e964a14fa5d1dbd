"""The allocation-free training entry point (mg_nn_gradient_static): through
the C ABI, its loss and gradient equal those of mg_nn_gradient with a
caller-allocated workspace on the same arguments (same kernels, same launch
shapes, fixed-order reductions: bit for bit), on two calls in a row, the
second with a smaller batch (so stale buffer contents of the first call
would show), with and without a box index; batches beyond its static limit
are rejected with MG_EINVAL."""
import numpy as np
import pytest
import torch

from oracle import nn_oracle as N
from paper_1708_08434_amd import mg as M
from paper_1708_08434_amd import nn as NN

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def params(seed):
    return N.init_params(seed).astype(np.float32)


def batch(seed, nbox):
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(rng.standard_normal((nbox, 10, 10, 10)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.standard_normal((nbox, 8, 8, 8)).astype(np.float32)).cuda()
    return x, t


def both(net, x, t, idx=None):
    nbox = int(idx.numel()) if idx is not None else int(x.shape[0])
    ip = 0 if idx is None else idx.data_ptr()
    ref_loss = net.gradient(x, t, idx=idx)
    ref_grad = net.get_grad()
    loss = NN.mg_nn_gradient_static(net.h, nbox, ip, x.data_ptr(), t.data_ptr())
    grad = net.get_grad()
    return ref_loss, ref_grad, loss, grad


@pytest.mark.parametrize("indexed", [False, True], ids=["plain", "indexed"])
def test_static_gradient_equals_workspace_gradient(indexed):
    net = NN.Net(params(5))
    for call, nbox in enumerate((NN.MG_NN_STATIC_MAX_BOXES, 9)):
        say("static gradient call", call, "nbox", nbox, "indexed", indexed)
        if indexed:
            x, t = batch(100 + call, nbox + 13)
            idx = torch.from_numpy(np.random.default_rng(7 + call).permutation(nbox + 13)[:nbox]
                                   .astype(np.int32)).cuda()
        else:
            x, t = batch(100 + call, nbox)
            idx = None
        ref_loss, ref_grad, loss, grad = both(net, x, t, idx)
        assert np.isfinite(ref_loss) and ref_loss > 0
        assert loss == ref_loss, (call, loss, ref_loss)
        assert np.array_equal(grad, ref_grad), (call, np.abs(grad - ref_grad).max())


def test_static_gradient_rejects_batches_beyond_its_limit():
    net = NN.Net(params(6))
    x, t = batch(3, NN.MG_NN_STATIC_MAX_BOXES + 1)
    for nbox in (NN.MG_NN_STATIC_MAX_BOXES + 1, 0):
        with pytest.raises(M.MGError) as e:
            NN.mg_nn_gradient_static(net.h, nbox, 0, x.data_ptr(), t.data_ptr())
        assert e.value.code == M.MG_EINVAL
    # the entry point still works after a rejected call
    x, t = batch(4, 3)
    ref_loss, ref_grad, loss, grad = both(net, x, t)
    assert loss == ref_loss and np.array_equal(grad, ref_grad)
