"""Host-side checks of bench.py that need no GPU: the algorithmic byte count
behind the roofline figure, and the refusal of more than one GPU."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_bytes_of_an_rk4_step():
    """Per RK4 step of an n^3 box: each of the 4 stages reads its stencil
    input once over the stored points, and the accumulator scheme moves 12
    pointwise arrays over the active points (stage 1 writes u1 and acc,
    stages 2 and 3 read u_n and acc and write u_s and acc, stage 4 reads acc
    and writes u_n), 25 float64 fields each."""
    b = _bench().alg_bytes_per_stage(256)
    stored, act, f = 262 ** 3, 256 ** 3, 25 * 8
    assert sum(b) == f * (4 * stored + 12 * act)
    assert b[0] == b[3] == f * (stored + 2 * act)
    assert b[1] == b[2] == f * (stored + 4 * act)
    assert abs(sum(b) / 4 / 1e9 - 13.663) < 1e-3  # the mean per launch quoted with the roofline
    assert abs(sum(b) / act - 3257.6) < 0.1       # bytes per zone cycle (about 3258)


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 2
    assert "one GPU" in out.stdout


def test_measured_traffic_belongs_to_the_committed_kernel():
    """The HBM traffic the bench line reports was counted on the kernel source
    that is committed (the figure is keyed by the source's SHA-256), with the
    headline tile and box, and fetched plus written bytes add up."""
    b = _bench()
    digest = b.kernel_source_digest()
    assert digest in b.MEASURED_TRAFFIC, "kernel source changed since the traffic counters were taken"
    m = b.MEASURED_TRAFFIC[digest]
    assert tuple(m["tile"]) == (8, 8, 8, 2, 1) and m["n"] == 256
    assert m["bytes_per_launch"] == m["fetch_bytes"] + m["write_bytes"]
    assert os.path.exists(os.path.join(ROOT, m["profile"]))
    with open(os.path.join(ROOT, m["profile"])) as f:
        assert digest[:16] in f.read()


def test_committed_tune_cache_covers_the_benchmark_workloads():
    """The committed tuning cache holds a shape for every benchmark workload
    (256^3 and 128^3 boxes and the equatorial half box in float64, 256^3 in
    mixed precision, the 9-box hierarchy in both), so the bench line takes
    its tiles from it instead of timing them."""
    import json
    with open(os.path.join(ROOT, "paper_2607_08743_amd", "tune_cache.jsonl")) as f:
        keys = {(e["arch"], e["precision"], e["nbox"], e["bucket"]) for e in map(json.loads, filter(str.strip, f))}
    for key in (("gfx950", 0, 1, 24), ("gfx950", 0, 1, 21), ("gfx950", 0, 1, 23), ("gfx950", 1, 1, 24),
                ("gfx950", 0, 9, 23), ("gfx950", 1, 9, 23)):
        assert key in keys, key
