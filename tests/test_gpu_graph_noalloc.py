"""The allocation-free advance captured in a HIP graph (needs a GPU).

fskmc_advance_noalloc enqueues kernel launches only, so a caller can record it
into a graph.  The call is made once eagerly (the library looks up its static
scratch on the first call on a device), then recorded with torch's graph
capture on the capturing stream and replayed three times; before each replay
the lattice is reset eagerly, and after each replay the lattice, the per-block
events and the event total must equal the eager call's."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_noalloc_replays_in_a_graph():
    from paper_1105_4673_amd import fskmc as F
    L, b, prm = 256, 16, (1.0, 1.0, 1.0, 0.0, 1.0)
    nb = (L // b) ** 2
    ctx = F.fskmc_ctx_create(0)
    try:
        sim = F.Sim(ctx, "flip", L, L, prm, b=b, n_colours=2, dt=0.1, T=10.0, split=1, seed=0, replica=9)
        sim.init(1, 0.5)
        lat0 = torch.from_numpy(sim.lattice().copy()).to("cuda")
        sim.close()
    finally:
        F.fskmc_ctx_destroy(ctx)
    lat = lat0.clone()
    w = torch.zeros(nb, dtype=torch.int32, device="cuda")
    ev = torch.zeros(1, dtype=torch.int64, device="cuda")

    def call(stream):
        F.fskmc_advance_noalloc(0, stream, 2, L, L, F.FSKMC_MODEL_FLIP, prm, b, b, 2, 0.1, 10.0, 1, 0, 9,
                                lat.data_ptr(), 0, 30, w.data_ptr(), ev.data_ptr())

    print("eager call", flush=True)
    call(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    want = (lat.cpu().numpy().copy(), w.cpu().numpy().copy(), int(ev.item()))
    assert want[2] > 0

    g = torch.cuda.CUDAGraph()
    lat.copy_(lat0)
    torch.cuda.synchronize()
    print("capture", flush=True)
    with torch.cuda.graph(g):
        call(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for rep in range(3):
        lat.copy_(lat0)
        w.fill_(-1)
        ev.fill_(-1)
        torch.cuda.synchronize()
        print(f"replay {rep}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        got = (lat.cpu().numpy(), w.cpu().numpy(), int(ev.item()))
        assert got[0].tobytes() == want[0].tobytes(), rep
        assert np.array_equal(got[1], want[1]) and got[2] == want[2], rep
