"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU needed): every HIP source is compiled for the host only, with the
sanitizers on the host side, and linked with tests/sanitize_abi_main.c, which
calls every entry point of include/rmdf.h along its argument-checking paths
and checks the returned status.  Any out-of-bounds access, use after free,
leak or undefined arithmetic on those paths aborts the run."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.mark.skipif(shutil.which("hipcc") is None or not os.path.exists(CLANG), reason="ROCm compilers not available")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all"]
    procs, objs = [], []
    for src in sorted(glob.glob(os.path.join(ROOT, "paper_1408_3526_amd", "csrc", "*.hip"))):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = ["hipcc", "--cuda-host-only", "-fgpu-rdc", "-O1", "-g", "-std=c++17", "-fPIC", *san, "-c", src, "-o", obj]
        procs.append((subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    for p, src in procs:
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, (src, err[-3000:])
    drv = str(tmp_path / "drv.o")
    subprocess.check_call([CLANG, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"), "-c",
                           os.path.join(ROOT, "tests", "sanitize_abi_main.c"), "-o", drv])
    exe = str(tmp_path / "abi_sanitized")
    r = subprocess.run(["hipcc", "-fgpu-rdc", "--offload-arch=gfx950", *san, *objs, drv, "-o", exe],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-4000:])
    assert "sanitized abi ok" in r.stdout, r.stdout[-3000:]
    assert "runtime error" not in r.stderr
