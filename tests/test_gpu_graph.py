"""The compute calls only enqueue kernels on the caller's stream (no
allocation, no memset, no synchronisation), so a forward + reconstruction
can be captured once in a HIP graph and replayed.  Every replay, with new
input data and eager work in between, must equal the eager result."""
import numpy as np
import pytest

from paper_1505_07690_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,level,L,dtype", [((64, 64, 64), 1, 16, "c64"), ((48, 40, 32), 0, 8, "bf16")],
                         ids=["64cube_plane_c64", "48x40x32_three_pass_bf16"])
def test_graph_replays_equal_eager(shape, level, L, dtype):
    import torch
    from paper_1505_07690_amd import os3d
    assert torch.cuda.is_available()
    n = inputs.icosahedral_orientations(level)
    bank = os3d.Bank(shape, n, os3d.make_params(L=L, s_theta=inputs.s_theta_for(len(n))))
    ws = bank.workspace()
    f = torch.empty(shape, dtype=torch.float32, device="cuda")
    is16 = dtype != "c64"
    U = torch.empty((len(n),) + shape, dtype=torch.int32 if is16 else torch.complex64, device="cuda")
    sc = torch.empty(len(n), dtype=torch.float32, device="cuda") if is16 else None
    rec = torch.empty(shape, dtype=torch.float32, device="cuda")
    vols = [torch.from_numpy(inputs.tubes(shape, 4, 1.5, 0.1, 0, 40 + k)).cuda() for k in range(4)]

    def run():
        os3d.forward(f, bank, dtype=dtype, ws=ws, out=U, scales=sc)
        os3d.reconstruct(U, bank, scales=sc, dtype=dtype, ws=ws, out=rec)

    f.copy_(vols[0])
    run()  # warm-up outside the capture (sets kernel attributes)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for k in range(4):
        f.copy_(vols[k])
        g.replay()
        torch.cuda.synchronize()
        got = rec.clone()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        run()
        torch.cuda.synchronize()
        assert torch.equal(got, rec), k
        assert np.isfinite(junk.item())
