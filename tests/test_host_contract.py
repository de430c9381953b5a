"""Host-side contract checks that need no GPU: the product path fails loudly
when the HIP library is missing (no CPU fallback), and the benchmark refuses
more than one GPU with a message."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(code_or_args, timeout=120):
    args = [sys.executable] + (["-c", code_or_args] if isinstance(code_or_args, str) else code_or_args)
    return subprocess.run(args, cwd=ROOT, capture_output=True, text=True, timeout=timeout)


def test_missing_library_raises_instead_of_falling_back():
    r = _run("from paper_1906_06060_amd import hotrg\n"
             "try:\n"
             "    hotrg.load('/nonexistent/libhotrg_gfx950.so')\n"
             "except hotrg.HotrgUnavailable as e:\n"
             "    print('unavailable:', e)\n"
             "else:\n"
             "    raise SystemExit('no error')\n")
    assert r.returncode == 0, r.stderr
    assert "unavailable:" in r.stdout


def test_bench_refuses_several_gpus():
    r = _run(["bench.py", "--gpus", "2"])
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
