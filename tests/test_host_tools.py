"""Host-only C++ checks, built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU, no HIP).

* the launch autotuner's search control (time budget, abandonment of
  candidates whose warm-up rules them out, progress bookkeeping) against a
  simulated clock with a many-mode cost model;
* the shared tree/plan header (Recall and fixed-block hit sets over every
  range of small trees, node ids, effective ranks, stitch workspace
  layouts), compiled for the host side only by hipcc (the header includes
  the HIP runtime header) with the sanitizers applied to host code.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_06647_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _build_and_run(src, tmp_path, hip=False):
    exe = str(tmp_path / os.path.basename(src).replace(".cpp", ""))
    if hip:
        if not os.path.exists(HIPCC):
            pytest.skip("needs hipcc")
        # host side only; every sanitizer flag is scoped to the host pass
        cmd = [HIPCC, "--cuda-host-only", "-x", "hip", "-std=c++17", "-O1", "-g",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all"]
    else:
        if shutil.which("g++") is None:
            pytest.skip("needs g++")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    cmd += ["-I" + CSRC, os.path.join(HOST, src), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    return out


def test_autotune_search_control(tmp_path):
    out = _build_and_run("tune_search_check.cpp", tmp_path)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr


def test_tree_plan_header_under_sanitizers(tmp_path):
    out = _build_and_run("common_check.cpp", tmp_path, hip=True)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr
