"""AddressSanitizer and UndefinedBehaviorSanitizer builds, run without a GPU: the oracle
on small cases of every entry point (oracle/sanitize_main.c), and the library's host
logic (paper_2509_21832_amd/csrc/sanitize_host_main.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    exe = tmp_path / "oracle_san"
    src = os.path.join(ROOT, "oracle")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fopenmp", "-I", src,
           os.path.join(src, "sanitize_main.c"), os.path.join(src, "mm_closure_oracle.c"), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "all cases completed" in r.stdout


HOST_SOURCES = ("mm_host.cpp", "mm_mlp.cpp")
KERNEL_OBJECTS = ("mm_kernels2d.o", "mm_fused2d.o", "mm_fused2d_lk.o", "mm_kernels1d.o", "mm_closure.o",
                  "mm_source.o")


@pytest.mark.slow
def test_host_logic_under_address_and_undefined_sanitizers(tmp_path):
    """The library's host code (configuration checks, time-step rule, argument checks of
    every entry point, context creation and its clean-up when the HIP runtime fails) built
    with AddressSanitizer and UndefinedBehaviorSanitizer on the host side only, linked with
    the kernel objects of the regular build, and driven without a GPU
    (paper_2509_21832_amd/csrc/sanitize_host_main.cpp)."""
    pkg = os.path.join(ROOT, "paper_2509_21832_amd")
    src, objdir = os.path.join(pkg, "csrc"), os.path.join(pkg, "_build")
    hipcc, clang = "/opt/rocm/bin/hipcc", "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("the ROCm compilers are not available")
    kobjs = [os.path.join(objdir, o) for o in KERNEL_OBJECTS]
    if not all(os.path.exists(o) for o in kobjs):
        pytest.skip("kernel objects missing: run __graft_entry__.build() first")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", src]
    # sanitizers on the host side of the HIP sources only; device code as in the regular build
    san_host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined"]
    objs = []
    for s in HOST_SOURCES:
        o = str(tmp_path / (os.path.splitext(s)[0] + ".o"))
        cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
               "-Wno-unused-value", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san_host + inc + \
              ["-x", "hip", "-c", os.path.join(src, s), "-o", o]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
        objs.append(o)
    # the host-logic program and the link: plain host C++ (no HIP source on these lines)
    main_o = str(tmp_path / "main.o")
    host_flags = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]
    subprocess.run([clang] + host_flags + inc + ["-c", os.path.join(src, "sanitize_host_main.cpp"), "-o", main_o],
                   check=True, capture_output=True, text=True)
    exe = str(tmp_path / "host_san")
    subprocess.run([clang, "-fsanitize=address,undefined", main_o] + objs + kobjs +
                   ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "all cases completed" in r.stdout
