"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the library is rebuilt with the sanitizers on its host code
(device code unchanged) and tests/asan/abi_driver.cpp calls every entry
point with arguments it must reject and with valid ones that need no GPU."""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_10129_amd", "csrc")
ROCM = "/opt/rocm"


def _runtime_dir():
    hits = glob.glob(os.path.join(ROCM, "lib", "llvm", "lib", "clang", "*", "lib", "linux",
                                  "libclang_rt.asan-x86_64.so"))
    return os.path.dirname(hits[0]) if hits else None


@pytest.mark.slow
def test_abi_host_code_under_sanitizers(tmp_path):
    rt = _runtime_dir()
    if rt is None or not os.path.exists(os.path.join(ROCM, "bin", "hipcc")):
        pytest.skip("no clang sanitizer runtime in this image")
    # every sanitizer flag applies to the host side only
    san = []
    for f in ("address", "undefined"):
        san += ["-Xarch_host", "-fsanitize=" + f]
    san += ["-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in sorted(os.listdir(CSRC)):
        if not src.endswith((".cpp", ".hip")):
            continue
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        subprocess.check_call([os.path.join(ROCM, "bin", "hipcc"), "-O1", "-g", "-std=c++17", "-fPIC",
                               "--offload-arch=gfx950", "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
                               "-packed-fp32-ops", *san, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj],
                              stderr=subprocess.DEVNULL)
        objs.append(obj)
    lib = str(tmp_path / "libctmi_san.so")
    subprocess.check_call([os.path.join(ROCM, "bin", "hipcc"), "--offload-arch=gfx950", "-shared", "-fPIC", *san,
                           "-Xarch_host", "-shared-libsan", "-o", lib, *objs], stderr=subprocess.DEVNULL)
    exe = str(tmp_path / "abi_driver")
    host_san = ["-fsanitize=" + f for f in ("address", "undefined")]
    subprocess.check_call([os.path.join(ROCM, "llvm", "bin", "clang++"), "-g", "-O1", "-std=c++17", *host_san,
                           "-fno-sanitize-recover=undefined", "-shared-libsan",
                           os.path.join(ROOT, "tests", "asan", "abi_driver.cpp"), lib, "-Wl,-rpath," + str(tmp_path),
                           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
                           "-o", exe])
    env = dict(os.environ, LD_LIBRARY_PATH=rt, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
