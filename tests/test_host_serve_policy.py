"""CPU test of the request server's admission policy (paper_1308_2445_amd/csrc/serve_policy.h,
the same header the server compiles): tests/serve_policy_harness.cpp runs unit cases and a
mock executor over request streams with more systems than slots, built with g++ plainly and
under AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1308_2445_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "serve_policy_harness.cpp")


@pytest.mark.parametrize("sanitize", [False, True])
def test_admission_policy_with_mock_executor(tmp_path, sanitize):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / ("serve_policy" + ("_san" if sanitize else "")))
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    subprocess.run([gxx, "-std=c++17", *flags, "-I", CSRC, HARNESS, "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    out = subprocess.run([exe], check=True, env=env, capture_output=True, text=True).stdout
    print(out)
    lines = out.strip().splitlines()
    assert lines[-1] == "ok"
    sims = [l for l in lines if l.startswith("simulation")]
    assert len(sims) == 4
    # the roomy stream rejects nothing; the one whose resident blocks outgrow the budget does
    assert "0 rejected" in sims[0] and "0 rejected" not in sims[2]
