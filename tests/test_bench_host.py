"""Host-side logic of bench.py (no GPU): the shipped launch lookup used by the profiling mode,
the guard that reports counter traffic only for the profiled source and launch, and the
n/precision sweep's case list."""
import ast
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


class _Hisq:
    """The one attribute of the binding these helpers read."""
    TUNING_PATH = os.path.join(ROOT, "paper_1409_1510_amd", "tuning", "gfx950.txt")
    HISQ_F64, HISQ_F32, HISQ_F16 = 0, 1, 2


def test_shipped_launch_reads_the_table():
    cfg = None
    for line in open(_Hisq.TUNING_PATH):
        f = line.split()
        if f and not f[0].startswith("#") and [int(v) for v in f[:8]] == [32, 32, 32, 8, 1, 18, 16, 0]:
            cfg = tuple(int(v) for v in f[8:13])
    assert cfg is not None
    assert bench.shipped_launch(_Hisq, (32, 32, 32, 8), 1, 18, 16, 0) == cfg
    # a lattice or size the table does not hold
    assert bench.shipped_launch(_Hisq, (8, 8, 8, 8), 1, 18, 16, 0) is None
    assert bench.shipped_launch(_Hisq, (32, 32, 32, 8), 1, 18, 63, 0) is None


def test_traffic_only_for_the_profiled_launch():
    fields = {}
    for line in open(bench.PROFILE_SUMMARY):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    cfg = ast.literal_eval(fields["launch_config"])
    assert bench.measured_traffic(cfg) == int(fields["hbm_bytes_per_launch"])
    other = (cfg[0] * 2 if cfg[0] < 4 else 1,) + tuple(cfg[1:])
    assert bench.measured_traffic(other) is None


def test_sweep_cases_cover_every_naik_format():
    cases = bench.sweep_cases(_Hisq)
    assert {(p, r) for p, r, _ in cases} == {(0, 18), (1, 18), (1, 14), (1, 13), (1, 9),
                                              (2, 18), (2, 14), (2, 9)}
    assert len({name for _, _, name in cases}) == len(cases)


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU: --gpus N > 1 exits with a message before touching a device."""
    import subprocess
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode != 0
    assert "one GPU" in (res.stdout + res.stderr)
