"""Host memory and undefined-behaviour checks (CPU only): the FP64 oracle's
C sources built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, -fno-sanitize-recover) run a standalone driver over every grid-level
entry point; and the host part of the C ABI (parameter validation, sizes,
the error paths of every entry point without a device) built with the same
sanitizers on its host side runs the ABI checks of a C driver (on a host
without a GPU every entry point's device work fails cleanly).  A sanitizer
report makes the driver exit nonzero."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _env():
    env = dict(os.environ)
    # verify_asan_link_order=0: the process environment may preload another
    # library ahead of the sanitizer runtime
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    return env


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off"] + SAN + [
        "-o", exe, os.path.join(HERE, "sanitize", "oracle_driver.c"),
        os.path.join(ROOT, "oracle", "cglbm_oracle.c"), os.path.join(ROOT, "oracle", "d2q9_oracle.c"),
        "-lm"]
    subprocess.check_call(cmd)
    r = subprocess.run([exe], env=_env(), capture_output=True, text=True, timeout=600)
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0 and "oracle driver: ok" in r.stdout, r.stderr[-4000:]


def test_c_abi_host_side_under_address_and_undefined_sanitizers(tmp_path):
    """The library built as usual (device code for gfx950, which this host
    without a GPU never runs) with the sanitizers on its host side, linked
    with a C driver of the ABI's validation and error paths."""
    from paper_2309_07801_amd import build as B
    if not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not found")
    objs, procs = [], []
    san = ["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all"]
    for u in B.UNITS:
        obj = str(tmp_path / (os.path.splitext(u)[0] + ".o"))
        objs.append(obj)
        cmd = [B.HIPCC] + B.FLAGS + san + ["-I", os.path.join(ROOT, "include"), "-c", "-o", obj,
                                             os.path.join(B.CSRC, u)]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-3000:]
    exe = str(tmp_path / "abi_driver")
    cmd = [B.HIPCC, "--offload-arch=gfx950", "-g", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-x", "c",
           os.path.join(HERE, "sanitize", "abi_driver.c"), "-x", "none"] + objs + ["-o", exe]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    env = _env()
    # the HIP runtime underneath is not instrumented: leak reports from it are
    # not the library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0 and "abi driver: ok" in r.stdout, r.stderr[-4000:]
