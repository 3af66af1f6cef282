"""The library's host logic under AddressSanitizer, without a GPU.

Every source is compiled host-only (no device code) with ASan, linked with a
host emulation of the HIP runtime calls it makes (tests/host_emulation), and
driven through every C-ABI entry point: planning, uploads, graph capture,
state save/restore, kernel timing and teardown.  Launches are checked against
the hardware's grid/block/LDS limits and counted, not executed.  Copies and
fills run only when their stream is synchronised, so a host buffer freed (or
a stack frame left) before its asynchronous copy has run is reported; the
benchmark's own call sequence (every workload's contexts created, run and
destroyed one after another) is replayed the same way.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_14046_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_emulation")
SOURCES = ["engine", "conv", "conv_f32", "conv_bf16", "conv_bf16x3", "norm", "jops", "ops", "dwconv", "pwconv", "se", "modules", "mnet"]
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and shutil.which("g++") and shutil.which("nm")),
                    reason="needs hipcc, g++ and nm")
def test_host_logic_under_address_sanitizer(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    procs, objs = [], []
    for s in SOURCES:
        o = str(tmp_path / (s + ".o"))
        objs.append(o)
        cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-O0", "-g", "-std=c++17", "-fPIC",
               "-Xarch_host", "-fsanitize=address", *inc, "-c", os.path.join(CSRC, s + ".hip"),
               "-o", o]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, out[-3000:]
    # code-object symbols referenced by the host-only objects
    und = subprocess.run(["nm", "-u", *objs], capture_output=True, text=True, check=True).stdout
    syms = sorted(set(re.findall(r"__hip_fatbin_[0-9a-f]+", und)))
    gen = tmp_path / "fatbins.cpp"
    gen.write_text('extern "C" {\n' + "".join("char %s[16];\n" % s for s in syms) + "}\n")
    rocm_inc = ["-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    exe = str(tmp_path / "emu")
    subprocess.run(["g++", "-O0", "-g", "-std=c++17", "-fsanitize=address", *inc, *rocm_inc,
                    os.path.join(HERE, "stubs.cpp"), os.path.join(HERE, "driver.cpp"), str(gen),
                    *objs, "-o", exe], check=True, capture_output=True)
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:detect_stack_use_after_return=1:abort_on_error=0")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-5000:])
    assert r.stdout.count("ok:") == 21
    assert "emulation errors: 0" in r.stdout
    r = subprocess.run([exe, "bench"], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-5000:])
    assert "ok: benchmark call sequence" in r.stdout and "emulation errors: 0" in r.stdout
