"""The serving loop on the GPU: every result is the same alone and in the
mix (concurrent streams, batched launches, 16-bit storage, the fused
processing path), a served job matches the oracle, and a tight HBM budget
serialises jobs without exceeding it."""
import numpy as np
import pytest

import oracle as O
from paper_1505_07690_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    from paper_1505_07690_amd import os3d
    os3d.lib()
    return t


def _alone(torch, vol, n, L, op, dtype):
    from paper_1505_07690_amd import os3d, serve
    bank = os3d.Bank(tuple(vol.shape), serve._orients(n), serve._params(n, L))
    if op == "process":
        out = os3d.process(vol, bank, "soft_threshold", 1.5)
    else:
        U, sc = os3d.forward(vol, bank, dtype=dtype)
        out = os3d.reconstruct(U, bank, scales=sc, dtype=dtype)
    torch.cuda.synchronize()
    return out


def test_alone_equals_mix(torch):
    from paper_1505_07690_amd.serve import Server
    jobs = [((128, 128, 128), 162, 16, "reconstruct", "c64"),
            ((128, 128, 128), 42, 16, "reconstruct", "c64"),
            ((64, 64, 64), 42, 16, "reconstruct", "c64"),
            ((64, 64, 64), 42, 16, "reconstruct", "c64"),
            ((96, 80, 64), 42, 24, "reconstruct", "c64"),
            ((64, 64, 64), 42, 16, "reconstruct", "c64"),
            ((32, 32, 32), 12, 8, "reconstruct", "bf16"),
            ((64, 64, 64), 162, 24, "process", "c64"),
            ((64, 64, 64), 42, 16, "reconstruct", "c64"),
            ((32, 32, 32), 12, 8, "reconstruct", "bf16")]
    vols = [inputs.tubes_device(sh, 12, (1.0, 3.0), 0.2, 0, 100 + i) for i, (sh, *_) in enumerate(jobs)]
    torch.cuda.synchronize()
    with Server(64 << 30, n_slots=2, max_batch=4) as s:
        futs = [s.submit(v, n, L, op=op, dtype=dt) for v, (sh, n, L, op, dt) in zip(vols, jobs)]
        outs = [f.result(timeout=120) for f in futs]
        st = s.stats()
    assert st["ok"] == len(jobs)
    assert st["max_batch"] > 1, st  # jobs that queued behind the first two shared launches
    for v, o, (sh, n, L, op, dt) in zip(vols, outs, jobs):
        assert tuple(o.shape) == sh
        assert torch.equal(o, _alone(torch, v, n, L, op, dt)), (sh, n, L, op, dt)


def test_16bit_jobs_at_256cube_on_concurrent_slots(torch):
    """bf16 and fp16 jobs on the two-pass 256^3 path (fp16 intermediates and
    persistent score passes for bf16) running on two slots at once, next to
    a complex64 one: every served result equals the same job run alone."""
    from paper_1505_07690_amd.serve import Server
    jobs = [((256, 256, 256), 42, 16, "reconstruct", "bf16"),
            ((256, 256, 256), 42, 16, "reconstruct", "c64"),
            ((256, 256, 256), 42, 16, "reconstruct", "bf16"),
            ((256, 256, 256), 42, 16, "reconstruct", "fp16"),
            ((128, 128, 128), 42, 16, "reconstruct", "bf16")]
    vols = [inputs.tubes_device(sh, 12, (1.0, 3.0), 0.2, 0, 200 + i) for i, (sh, *_) in enumerate(jobs)]
    torch.cuda.synchronize()
    with Server(64 << 30, n_slots=2, max_batch=1) as s:
        futs = [s.submit(v, n, L, op=op, dtype=dt) for v, (sh, n, L, op, dt) in zip(vols, jobs)]
        outs = [f.result(timeout=120) for f in futs]
        st = s.stats()
    assert st["ok"] == len(jobs)
    for v, o, (sh, n, L, op, dt) in zip(vols, outs, jobs):
        assert torch.equal(o, _alone(torch, v, n, L, op, dt)), (sh, n, L, op, dt)


def test_served_job_matches_oracle(torch):
    from paper_1505_07690_amd.serve import Server
    shape = (32, 32, 32)
    v = inputs.tubes_device(shape, 12, (1.0, 3.0), 0.2, 0, 7)
    with Server(8 << 30, n_slots=2) as s:
        got = s.submit(v, 42, 16).result(timeout=60).cpu().numpy()
    f = v.cpu().numpy().astype(np.float64)
    n = inputs.icosahedral_orientations(1)
    ob = O.build_bank(shape, n, O.WaveletParams(L=16, s_theta=inputs.s_theta_for(42)))
    want = O.reconstruct(O.forward(f, ob), ob)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-5


def test_tight_budget_serialises(torch):
    from paper_1505_07690_amd import os3d, serve
    from paper_1505_07690_amd.serve import Server
    shape = (64, 64, 64)
    ex = serve.GpuExecutor(n_slots=3)
    key = (shape, 42, 16)
    bank_b = ex.bank_bytes(key)
    bank = os3d.Bank(shape, serve._orients(42), serve._params(42, 16))
    one = ex.job_bytes(key, bank, 1, "reconstruct", "c64")
    assert ex.job_bytes_estimate(key, 1, "reconstruct", "c64") <= one  # the pre-bank check is a lower bound
    # one bank and one job (scores, volumes, workspace), not two jobs
    budget = bank_b + one + (2 << 20)
    vols = [inputs.tubes_device(shape, 12, (1.0, 3.0), 0.2, 0, 200 + i) for i in range(4)]
    with Server(budget, n_slots=3, max_batch=1, executor=ex) as s:
        outs = [s.submit(v, 42, 16) for v in vols]
        outs = [f.result(timeout=60) for f in outs]
        st = s.stats()
    assert st["ok"] == 4 and st["peak_bytes"] <= budget
    for v, o in zip(vols, outs):
        U, _ = os3d.forward(v, bank)
        assert torch.equal(o, os3d.reconstruct(U, bank))


def test_result_consumed_on_the_callers_stream_survives_later_jobs(torch):
    """A result is handed over to the stream it was submitted from: work the
    caller queues there on it (behind a 50 ms spin) still reads the right
    values after the caller drops the tensor and later jobs of the same
    shape allocate their outputs."""
    from paper_1505_07690_amd.serve import Server
    shape = (64, 64, 64)
    vols = [inputs.tubes_device(shape, 12, (1.0, 3.0), 0.2, 0, 300 + i) for i in range(5)]
    torch.cuda.synchronize()
    want = _alone(torch, vols[0], 42, 16, "reconstruct", "c64")
    with Server(16 << 30, n_slots=2, max_batch=1) as s:
        out = s.submit(vols[0], 42, 16).result(timeout=60)
        consumed = torch.empty_like(want)
        torch.cuda._sleep(120_000_000)  # bounded spin on the caller's stream
        consumed.copy_(out)
        del out
        outs = [s.submit(v, 42, 16).result(timeout=60) for v in vols[1:]]
        torch.cuda.synchronize()
    assert torch.equal(consumed, want)
    for v, o in zip(vols[1:], outs):
        assert torch.equal(o, _alone(torch, v, 42, 16, "reconstruct", "c64"))
