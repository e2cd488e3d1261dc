"""The allocation-free gradient entry point (pdnqp_mlp_gradient_noalloc):
on device buffers owned by the caller, with its partials in the library's
static scratch array, it returns the gradient and loss of the allocating
entry point pdnqp_mlp_gradient bit for bit -- on two calls in a row, the
second with fewer samples (the scratch keeps the first call's partials) --
and rejects sizes beyond its maximum."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_19557_amd as P
    P.load()
    return P


def _case(count, seed):
    rng = np.random.default_rng(seed)
    theta = (rng.standard_normal(5443) * 0.2).astype(np.float32)
    X = rng.standard_normal((count, 16)).astype(np.float32)
    Y = rng.standard_normal((count, 3)).astype(np.float32)
    return theta, X, Y


def test_noalloc_gradient_matches_allocating_entry_point(P):
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    for count, seed in ((3000, 1), (517, 2)):
        theta, X, Y = _case(count, seed)
        g_ref, loss_ref = P.mlp_gradient(theta, X, Y)
        th_d = torch.from_numpy(theta).cuda()
        x_d = torch.from_numpy(X).cuda()
        y_d = torch.from_numpy(Y).cuda()
        g_d = torch.full((5443,), float("nan"), dtype=torch.float32, device="cuda")
        l_d = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        P.mlp_gradient_noalloc(th_d.data_ptr(), x_d.data_ptr(), y_d.data_ptr(), count,
                               g_d.data_ptr(), l_d.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        g = g_d.cpu().numpy()
        assert np.array_equal(g, g_ref), (count, np.abs(g - g_ref).max())
        assert l_d.item() == loss_ref
    # loss pointer may be omitted
    P.mlp_gradient_noalloc(th_d.data_ptr(), x_d.data_ptr(), y_d.data_ptr(), count,
                           g_d.data_ptr(), None, stream.cuda_stream)
    torch.cuda.synchronize()
    assert np.array_equal(g_d.cpu().numpy(), g_ref)


def test_noalloc_gradient_rejects_sizes_beyond_its_maximum(P):
    import torch
    th = torch.zeros(5443, dtype=torch.float32, device="cuda")
    x = torch.zeros((1, 16), dtype=torch.float32, device="cuda")
    g = torch.zeros(5443, dtype=torch.float32, device="cuda")
    for count in (0, 16385):
        with pytest.raises(P.PdnqpError, match="count must be in"):
            P.mlp_gradient_noalloc(th.data_ptr(), x.data_ptr(), x.data_ptr(), count,
                                   g.data_ptr(), None, None)
