"""The admission scheduler (csrc/hs_sched.h, host logic only) under the
sanitizers: a multi-threaded submit / cancel / batch / complete stress
(tests/native/sched_stress.cpp) built with g++ and AddressSanitizer +
UndefinedBehaviorSanitizer, and again with ThreadSanitizer; each build must
run clean and pass its own invariant checks."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "sched_stress.cpp")

BUILDS = {
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"],
    "tsan": ["-fsanitize=thread"],
}


@pytest.mark.parametrize("kind", sorted(BUILDS))
def test_scheduler_stress_under_sanitizer(kind, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / f"sched_stress_{kind}")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread"] + BUILDS[kind] + [SRC, "-o", exe]
    subprocess.run(cmd, check=True)
    env = dict(os.environ)
    # other preloaded libraries may precede the sanitizer runtime
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:verify_asan_link_order=0"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sched_stress ok" in r.stdout
