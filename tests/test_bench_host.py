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
