"""The plain fill and the EA generation step captured in a HIP graph
(torch.cuda.graph): they allocate nothing and issue no memset, so a captured
launch sequence replays the eager results.  Every replay is checked against
the eager run, with eager work and synchronisations between replays."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_fill_and_ea_step_replay_from_a_graph(ctx, zg):
    n_per, ns = 4096, 96
    out = torch.empty(n_per * ns, dtype=torch.float64, device="cuda")
    f32 = torch.empty(n_per * ns, dtype=torch.float32, device="cuda")
    pop, genes = 2048, 300
    g = torch.Generator().manual_seed(3)
    P = (torch.rand((pop, genes), generator=g, dtype=torch.float64) * 4 - 2).cuda()
    F = (P * P).sum(dim=1)
    C = torch.empty_like(P)
    W = torch.empty(pop, dtype=torch.int32, device="cuda")

    def work():
        ctx.zg_fill_streams(out, n_per, ns, seed=7, stream0=5)
        ctx.zg_fill_streams(f32, n_per, ns, seed=8, stream0=6)
        ctx.zg_ea_step(P, F, C, W, tournament=3, rate=0.2, sigma=0.3, lo=-2.0, hi=2.0, seed=11,
                       stream=40, generation=2)

    work()
    torch.cuda.synchronize()
    ref = [out.cpu().numpy().tobytes(), f32.cpu().numpy().tobytes(), C.cpu().numpy().tobytes(),
           W.cpu().numpy().tobytes()]
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        work()   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        work()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in (out, f32, C):
            t.fill_(float("nan"))
        W.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [out.cpu().numpy().tobytes(), f32.cpu().numpy().tobytes(), C.cpu().numpy().tobytes(),
               W.cpu().numpy().tobytes()]
        for name, a, b in zip(("fill f64", "fill f32", "ea children", "ea winners"), got, ref):
            assert a == b, (rep, name)
        # eager work between replays
        ctx.zg_fill_streams(out, n_per, 8, seed=99)
        torch.cuda.synchronize()
    assert ctx.zg_error_flags() == 0
