"""The host code of the C ABI under AddressSanitizer (CPU only): the library
is rebuilt with the sanitizer on its host code (device code unchanged) and
test_abi.py runs against it in a child process with the sanitizer runtime
preloaded.  Every call there that needs no device (planning, argument
validation, error reporting, the BFP size query) then runs instrumented; a
heap overflow, use-after-free or similar error aborts the child."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_30128_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _runtime():
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.fixture(scope="module")
def asan_lib(tmp_path_factory):
    rt = _runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("no hipcc or no AddressSanitizer runtime")
    from paper_2605_30128_amd import build as hipbuild
    out = tmp_path_factory.mktemp("asan")
    flags = [f for f in hipbuild.FLAGS if f != "-O3"] + ["-O1", "-g"]
    host_asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs, procs = [], []
    for src in hipbuild.SOURCES:
        obj = str(out / (os.path.splitext(src)[0] + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *flags, *host_asan, "-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        log = p.communicate()[0]
        assert p.returncode == 0, log[-4000:]
    lib = str(out / "libchfsi_asan.so")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", lib, "-L/opt/rocm/lib",
                        "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return lib, rt


def test_abi_under_address_sanitizer(asan_lib):
    lib, rt = asan_lib
    env = dict(os.environ, CHFSI_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout
    assert "AddressSanitizer" not in r.stdout + r.stderr
