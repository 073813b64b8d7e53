"""The synthetic generator under AddressSanitizer and UndefinedBehaviorSanitizer.

The batched workload generates twelve stations; a driver (synth_driver.c)
runs slices of all twelve from twelve host threads at once (each call opens
its own OpenMP team, as concurrent calls from a thread pool would) and
compares them with a single-threaded run.  The sanitizers stop the run at
the first invalid access, leak or undefined operation.  CPU only.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_generator_twelve_stations_concurrently_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "synth_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "synth", "synth.c"), os.path.join(HERE, "synth_driver.c"),
           "-lpthread", "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1", OMP_NUM_THREADS="4",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, "100000"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "synth_driver ok" in r.stdout
