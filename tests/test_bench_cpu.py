"""The measurement plumbing of bench.py that runs without a GPU: the one-GPU
guard, the traffic calibration lookup and its source digest, and the
algorithmic flop counts of the processing kernels.  CPU only."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_calibration_is_keyed_by_the_kernel_sources():
    """The committed rocprofv3 calibration is keyed by a digest of the kernel
    sources: a lookup under its own digest finds the kernel, a lookup under
    another digest (kernels changed since the counters were taken) gives
    None, and the bench line then reports traffic as null."""
    b = _bench()
    digest = b.kernel_source_digest()
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        t = json.load(f)
    got = b.load_traffic("rec_first_load_scores", t["source_digest"])
    assert got is not None and got > 0
    assert b.load_traffic("rec_first_load_scores", "0" * 16) is None
    assert b.load_traffic("no_such_kernel", t["source_digest"]) is None
    if digest != t["source_digest"]:
        assert b.load_traffic("rec_first_load_scores", digest) is None


def test_processing_flop_counts():
    """5 log2 n flops per point of a length-n DFT: at 256^3 each direction's
    transform is split 12 + 12 radix-2 levels between the frequency and the
    natural side; on 128^2 planes the plane DFT has 14 levels."""
    b = _bench()
    assert b.process_flops_per_pair_voxel((256, 256, 256), "fwd_last_store_scores") == 2 * 60 + b.PHI_FLOPS
    assert b.process_flops_per_pair_voxel((256, 256, 256), "fwd_first_mul_bank") == 62
    assert b.process_flops_per_pair_voxel((128, 128, 128), "fwd_last_store_scores") == 2 * 70 + b.PHI_FLOPS
    assert b.process_flops_per_pair_voxel((128, 128, 128), "rec_last_accumulate") == 5 * 7 + 4
    assert b.process_flops_per_pair_voxel((48, 40, 32), "fwd_last_store_scores") is None


def test_step_flop_counts():
    """Forward + reconstruction: 5 log2 V flops per voxel-orientation for the
    transforms with antipodal pairs (one DFT per pair in each direction),
    twice that without, plus 6 for the multiply and the orientation sum:
    126 and 246 at 256^3; the FP32 fraction is the achieved rate over
    157.3 TFLOP/s."""
    b = _bench()
    V = 1 << 24
    assert b.step_flops(V, 162, True) == 126 * V * 162
    assert b.step_flops(V, 162, False) == 246 * V * 162
    assert b.step_flops(1 << 21, 42, True) == (5 * 21 + 6) * (1 << 21) * 42
    f = b.flops_figures(157.3e12 * 2e-3, 2.0)  # 2 ms of work at the peak rate
    assert abs(f["achieved_tflops"] - 157.3) < 1e-9 and abs(f["fp32_vector_frac"] - 1.0) < 1e-12
