"""The single-image path recorded into a HIP graph through torch.cuda.graph: prologue,
tables, fused query, training query, residual backward and the end-to-end RGB call.  Every
replay is compared with the eager result, with the program's own eager work and
synchronisations between replays (no entry point records a memset node)."""
import numpy as np
import pytest
import torch

import paper_2102_01289_amd as tm
from _cases import rgb_case, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["c32x2", "f64"])
def test_forward_and_backward_graph_replays(prec):
    H, W = 150, 230
    rgb = to_dev(rgb_case(H, W, 6, seed=17))
    g = to_dev(np.random.default_rng(2).standard_normal((H, W)).astype(np.float32))
    p = tm.make_params(5, 5, eps=0.1, H=H, W=W)
    m = tm.ToneMapper(H, W, p, prec)
    # eager reference (also allocates every lazily created buffer before capture)
    m.run_train(rgb)
    gv, gp = (t.clone() for t in m.backward_resid(g))
    L_ref = m.out.clone()
    rgb_ref = m.run_rgb(rgb).clone()
    torch.cuda.synchronize()

    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        m.run_train(rgb, stream=s)
        m.backward_resid(g, stream=s)
        m.query_rgb(rgb, 0.6, stream=s)
    for rep in range(4):
        m.out.zero_()
        m.grad_v.zero_()
        m.rgb_out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(m.out, L_ref), rep
        assert torch.equal(m.grad_v, gv), rep
        assert torch.equal(m.grad_params, gp), rep
        assert torch.equal(m.rgb_out, rgb_ref), rep
        _ = torch.randn(4096, device="cuda").sum().item()   # eager work between replays
    # the graph reads its inputs at replay time
    rgb.mul_(4.0)
    graph.replay()
    torch.cuda.synchronize()
    fresh = tm.ToneMapper(H, W, p, prec).run(rgb)
    torch.cuda.synchronize()
    assert torch.equal(m.out, fresh)


@pytest.mark.parametrize("recompute", [True, False])
def test_autograd_forward_backward_graph_capture(recompute):
    # The autograd Function passes eps, min L_d and max L_d to the kernels in device memory,
    # so its forward and backward make no host synchronisation and record into one graph
    # (torch's whole-network capture recipe: warm-up on a side stream, grads None before
    # capture).  Every replay equals the eager pass; new scalar values take effect on replay.
    from paper_2102_01289_amd.autograd import tonemap_luminance
    from _cases import lum_ref
    H, W = 96, 120
    lum = to_dev(lum_ref(rgb_case(H, W, 5, seed=31)))
    x = lum.clone().requires_grad_(True)
    eps = torch.tensor(0.1, device="cuda", requires_grad=True)
    lo = torch.tensor(0.0, device="cuda", requires_grad=True)
    hi = torch.tensor(1.0, device="cuda", requires_grad=True)
    g = to_dev(np.random.default_rng(5).standard_normal((H, W)).astype(np.float32))
    leaves = (x, eps, lo, hi)

    def step():
        L = tonemap_luminance(x, eps, lo, hi, n_bins=5, n_scales=4, recompute=recompute)
        L.backward(g)
        return L

    L_ref = step().detach().clone()
    grads_ref = [t.grad.clone() for t in leaves]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            for t in leaves:
                t.grad = None
            step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for t in leaves:
        t.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        L_static = step()
    for rep in range(4):
        L_static.zero_()
        for t in leaves:
            t.grad.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(L_static, L_ref), rep
        for t, r in zip(leaves, grads_ref):
            assert torch.equal(t.grad, r), rep
        _ = torch.randn(4096, device="cuda").sum().item()   # eager work between replays
    # a new eps read at replay time, without capturing again
    with torch.no_grad():
        eps.fill_(0.25)
    graph.replay()
    torch.cuda.synchronize()
    x2 = lum.clone().requires_grad_(True)
    e2 = torch.tensor(0.25, device="cuda", requires_grad=True)
    L2 = tonemap_luminance(x2, e2, lo.detach(), hi.detach(), n_bins=5, n_scales=4,
                           recompute=recompute)
    L2.backward(g)
    torch.cuda.synchronize()
    assert torch.equal(L_static, L2.detach())
    assert torch.equal(x.grad, x2.grad) and torch.equal(eps.grad, e2.grad)
