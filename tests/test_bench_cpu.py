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
