"""bench.py on the CPU: the one-GPU contract (more than one GPU is refused
with a JSON message and exit status 2, before any GPU work) and the traffic
figure's tie to the kernel source it was measured on."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_traffic_profile_matches_kernel_source():
    """The committed HBM-traffic counters are used only while they belong to the
    current sweep-kernel source (SHA-256) and to the kernel the bench times,
    else the bench reports null."""
    sys.path.insert(0, ROOT)
    import bench
    prof = json.load(open(os.path.join(ROOT, "profiles", "sweep_pass_cfg3_traffic.json")))
    src = open(os.path.join(ROOT, "paper_2011_02991_amd", "csrc", "sweep_kernels.hip"), "rb").read()
    same = prof["kernel_sha256"] == hashlib.sha256(src).hexdigest() and prof.get("kernel") == "k_sweep_reg_real_exact"
    t = bench.traffic_per_launch(bench.sweep_kernel_name("c64", 0, 1))
    assert (t is not None) == same
    assert bench.traffic_per_launch("k_sweep_reg_states") is None
    if same:
        assert abs(t - prof["bytes_per_launch"]) <= 1e-6 * prof["bytes_per_launch"]
