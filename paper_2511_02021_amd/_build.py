"""In-tree native builds: the host input generator (g++) and the HIP library
libnhdc for gfx950 (hipcc).  Each call recompiles; callers that only load a
library use ``lib_path`` and build only when nothing is there."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")

INPUTS_SO = os.path.join(PKG, "inputs", "libnhinputs.so")
NHDC_SO = os.path.join(PKG, "libnhdc.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)


def build_inputs():
    src = os.path.join(PKG, "inputs", "csrc")
    tmp = INPUTS_SO + ".tmp"
    _run(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-I", INCLUDE, "-I", src,
          os.path.join(src, "nhgrid.cpp"), os.path.join(src, "nhcase.cpp"), "-o", tmp])
    os.replace(tmp, INPUTS_SO)
    return INPUTS_SO


def nhdc_sources():
    src = os.path.join(PKG, "csrc")
    return sorted(os.path.join(src, f) for f in os.listdir(src) if f.endswith((".hip", ".cpp")))


def build_nhdc():
    src = os.path.join(PKG, "csrc")
    tmp = NHDC_SO + ".tmp"
    flags = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
             # packed FP32 forms stay off: plain float code only
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", src]
    _run([HIPCC] + flags + nhdc_sources() + ["-o", tmp])
    os.replace(tmp, NHDC_SO)
    return NHDC_SO


def ensure(path, builder):
    if not os.path.exists(path):
        builder()
    return path
