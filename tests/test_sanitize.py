"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Every csrc/*.hip source is compiled for the host alone with the sanitizers (no device code; each
translation unit's device-code bundle is replaced by an empty one, so nothing can be launched),
linked into a shared library, and tests/abi_sanitize.c drives the C ABI through it: argument
validation, workspace sizes, plan queries, backward layouts, batch-plan validation.  The sanitizers
abort the test program on an out-of-bounds access, a use after free or undefined behaviour.
"""
import concurrent.futures as cf
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_14258_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

# host-side instrumentation only (each -fsanitize= applies to the host pass)
HOST_FLAGS = ["-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer", "-Wno-unused-result"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not found")
def test_abi_under_address_and_undefined_sanitizers(tmp_path):
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [str(tmp_path / (os.path.basename(s)[:-4] + ".o")) for s in srcs]
    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda so: _run([HIPCC, *HOST_FLAGS, "-c", so[0], "-o", so[1]]), zip(srcs, objs)))
    # the device-code bundle each translation unit registers at load time: an empty one
    syms = set()
    for o in objs:
        syms.update(re.findall(r"(__hip_fatbin_[0-9a-f]+)", _run(["nm", "-u", o]).stdout))
    stub = tmp_path / "bundles.c"
    stub.write_text("".join('__attribute__((aligned(4096))) const char %s[32] = "__CLANG_OFFLOAD_BUNDLE__";\n' % s
                            for s in sorted(syms)))
    _run([CLANG, "-c", "-fPIC", str(stub), "-o", str(tmp_path / "bundles.o")])
    lib = tmp_path / "libldbp_san.so"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, str(tmp_path / "bundles.o"),
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", str(lib)])
    exe = tmp_path / "abi_sanitize"
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          os.path.join(ROOT, "tests", "abi_sanitize.c"), str(lib), f"-Wl,-rpath,{tmp_path}", "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "abi_sanitize: ok" in r.stdout, r.stdout + r.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)
