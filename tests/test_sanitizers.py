"""AddressSanitizer + UndefinedBehaviorSanitizer runs on the CPU:

- the FP64 oracle (oracle/nnref.c) on small periodic and cluster inputs,
  through every exported function (tests/sanitize/oracle_driver.c, gcc);
- the host side of the C ABI (csrc/api.hip compiled with the sanitizers on
  its host pass only) through descriptor and workspace sizes and every
  argument check that returns before a launch (tests/sanitize/abi_driver.c;
  no GPU is needed, no kernel is launched).

Each driver exits 0 and the sanitizers print nothing on a clean run."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math", "-ffp-contract=off",
                    "-fopenmp", *SAN_FLAGS, "-Wall", "-Wno-unused-function",
                    os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"], check=True)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "2"})
    assert "periodic:" in out and "cluster:" in out


def test_abi_host_paths_under_asan_ubsan(tmp_path):
    objs = [o for o in glob.glob(os.path.join(ROOT, "paper_2305_11805_amd", "_build", "*.o"))
            if not o.endswith("api.hip.o")]
    if not objs or not shutil.which("hipcc"):
        pytest.skip("needs hipcc and the objects of a library build")
    from paper_2305_11805_amd import build as nnbuild
    api_o = str(tmp_path / "api_san.o")
    host_san = []
    for f in SAN_FLAGS:  # the host pass only: each option directly after -Xarch_host
        host_san += ["-Xarch_host", f]
    flags = [f for f in nnbuild.CFLAGS if f != "-O3"] + ["-O1", "-g"]
    subprocess.run(["hipcc", *flags, *host_san, "-c", os.path.join(ROOT, "paper_2305_11805_amd", "csrc", "api.hip"),
                    "-o", api_o], check=True, capture_output=True)
    drv_o = str(tmp_path / "abi_driver.o")
    subprocess.run(["gcc", "-O1", "-g", *SAN_FLAGS, "-I", os.path.join(ROOT, "include"), "-c",
                    os.path.join(SAN, "abi_driver.c"), "-o", drv_o], check=True)
    exe = str(tmp_path / "abi_san")
    subprocess.run(["g++", *SAN_FLAGS, drv_o, api_o, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib", "-o", exe], check=True)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
    assert "abi host paths" in out
