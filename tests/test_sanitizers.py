"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, gcc) runs every entry point on small tori without a
report; the driver also checks identities the oracle must keep."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "oracle"),
           os.path.join(ROOT, "tests", "sanitize_oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stderr[-4000:]
    assert run.stdout.strip() == "ok"


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_library_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The product library with its host code instrumented (device code is
    built as usual, for gfx950) runs its host-only entry points -- schedules,
    thresholds, generated weights, argument checks -- without a report."""
    import concurrent.futures

    hipcc = "/opt/rocm/bin/hipcc"
    csrc = os.path.join(ROOT, "paper_2505_18508_amd", "csrc")
    # sanitizers on the host pass only: each -fsanitize= right after -Xarch_host
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-I" + csrc] + host_san
    srcs = sorted(f for f in os.listdir(csrc) if f.endswith(".hip"))

    def compile_one(f):
        obj = str(tmp_path / (f + ".o"))
        r = subprocess.run([hipcc] + common + ["-c", os.path.join(csrc, f), "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_asan")
    r = subprocess.run([hipcc, "--offload-arch=gfx950"] + host_san[:4] + ["-I" + os.path.join(ROOT, "include"),
                        "-x", "c", os.path.join(ROOT, "tests", "sanitize_host_driver.c"), "-x", "none"] + objs +
                       ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    # leaks are not checked: the HIP runtime keeps allocations until exit
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stderr[-4000:]
    assert run.stdout.strip() == "ok"
