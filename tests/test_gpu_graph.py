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
