"""The gradient pass of the closure network without a caller workspace
(wlb_mlp_grad_noalloc, for callers that cannot allocate device memory)
against the workspace version (wlb_mlp_grad) through the C ABI: the same
kernels on the same inputs must give the same gradient and loss bit for
bit.  Two calls in a row, the second with a smaller minibatch, check that
what the first call leaves in the library's fixed scratch array does not
leak into the second; a minibatch above the array's limit is refused."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

wlb = pytest.importorskip("paper_1909_13772_amd.wlb", reason="libwlb.so not built")
torch = pytest.importorskip("torch")


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    raw = np.empty((n, 7), np.float32)
    raw[:, :6] = rng.normal(0, 2e-3, (n, 6))
    raw[:, 6] = rng.normal(0, 5e-3, n)
    t = rng.uniform(0.0, 0.05, n).astype(np.float32)
    P = rng.normal(0, 0.3, wlb.MLP_NPARAM).astype(np.float32)
    P[:7] = 0.0
    P[7:14] = [400.0] * 6 + [150.0]
    return P, raw, t


def _grad(fn, n, seed):
    dev = torch.device("cuda")
    P, raw, t = _inputs(n, seed)
    Pd, rd, td = torch.tensor(P, device=dev), torch.tensor(raw, device=dev), torch.tensor(t, device=dev)
    g = torch.full((wlb.MLP_NPARAM,), float("nan"), dtype=torch.float32, device=dev)
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    if fn == "workspace":
        wsb = wlb.wlb_mlp_grad_workspace(n)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        wlb.wlb_mlp_grad(Pd.data_ptr(), rd.data_ptr(), td.data_ptr(), n, 40.0, g.data_ptr(), loss.data_ptr(),
                         ws.data_ptr(), wsb, s.cuda_stream)
    else:
        wlb.wlb_mlp_grad_noalloc(Pd.data_ptr(), rd.data_ptr(), td.data_ptr(), n, 40.0, g.data_ptr(), loss.data_ptr(),
                                 s.cuda_stream)
    s.synchronize()
    return g.cpu().numpy(), float(loss.cpu()[0])


def test_noalloc_gradient_matches_workspace_version_twice():
    # first a large minibatch (ragged tail), then a smaller one
    for n, seed in ((200003, 1), (4099, 2)):
        say(f"case mlp grad noalloc n={n}")
        g_ref, l_ref = _grad("workspace", n, seed)
        g_new, l_new = _grad("noalloc", n, seed)
        say(f"noalloc n={n}: loss {l_new:.6e} vs {l_ref:.6e}, max |dg| {np.abs(g_new - g_ref).max():.3e}")
        assert np.isfinite(g_ref).all() and np.isfinite(l_ref)
        assert np.array_equal(g_new, g_ref)
        assert l_new == l_ref


def test_noalloc_rejects_oversized_minibatch():
    say("case mlp grad noalloc limit")
    dev = torch.device("cuda")
    x = torch.zeros(16, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    with pytest.raises(wlb.WlbError) as e:
        wlb.wlb_mlp_grad_noalloc(x.data_ptr(), x.data_ptr(), x.data_ptr(), wlb.MLP_NOALLOC_MAX_SAMPLES + 1, 1.0,
                                 x.data_ptr(), x.data_ptr(), s.cuda_stream)
    assert e.value.code == wlb.WLB_ERR_ARG
    with pytest.raises(wlb.WlbError):
        wlb.wlb_mlp_grad_noalloc(x.data_ptr(), x.data_ptr(), x.data_ptr(), 0, 1.0, x.data_ptr(), x.data_ptr(),
                                 s.cuda_stream)
