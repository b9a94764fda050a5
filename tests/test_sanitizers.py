"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only,
no GPU): the oracle (valid, garbage and encoded frames, rANS coding
of frames and rejection of malformed coded data) and the host side of
libtmd (tables, messages, argument checks, plan creation without a GPU).
Any report aborts the child process.  The oracle's sanitized results must
equal those of its normal build."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_lib(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()


def test_oracle_under_sanitizers(tmp_path):
    so = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-shared", "-fPIC",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", so, os.path.join(ROOT, "oracle", "tmd_oracle.c"),
                    os.path.join(ROOT, "oracle", "rans_oracle.c"), "-lm"], check=True)
    script = os.path.join(HERE, "run_oracle.py")
    env = dict(os.environ, TMD_ORACLE_LIB=so, LD_PRELOAD=_gcc_lib("libasan.so"), **SAN_ENV)
    san = subprocess.run([sys.executable, script], env=env, capture_output=True, text=True, timeout=600)
    assert san.returncode == 0, san.stderr[-4000:]
    env.pop("TMD_ORACLE_LIB"), env.pop("LD_PRELOAD")
    ref = subprocess.run([sys.executable, script], env=env, capture_output=True, text=True, timeout=600)
    assert ref.returncode == 0, ref.stderr[-4000:]
    assert san.stdout.splitlines() == ref.stdout.splitlines()
    assert len(san.stdout.splitlines()) == 9


def test_library_host_code_under_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2411_02206_amd import build as lb
    so = str(tmp_path / "libtmd_san.so")
    flags = [f for f in lb.FLAGS if f not in ("-O3",)]
    # host code instrumented, device code as usual
    subprocess.run([lb.HIPCC, *flags, "-O1", "-g", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                    "-o", so, lb.SRC], check=True, capture_output=True)
    exe = str(tmp_path / "abi_host")
    subprocess.run(["/opt/rocm/llvm/bin/clang", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    f"-I{os.path.join(ROOT, 'include')}", "-o", exe, os.path.join(HERE, "abi_host.c"), so,
                    f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    env = dict(os.environ, HIP_VISIBLE_DEVICES="", **SAN_ENV)
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-4000:])
