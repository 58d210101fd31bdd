"""Build the engine's shared library (libnufold.so) in-tree for gfx950."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnufold.so")
SOURCES = ["engine.hip", "fold.hip", "tail.hip", "mlp.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose=False):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libnufold.so")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


# AddressSanitizer and UndefinedBehaviorSanitizer on the host pass only (the
# device code is built as usual, at -O1 to keep the build short): the JSON
# reader, the schema checks and the plan build run under the sanitizers when
# a host program calls nf_create (without a GPU it returns NF_EDEVICE after
# the plan build).
SANITIZE_FLAGS = [
    f"--offload-arch={ARCH}", "-O1", "-std=c++17", "-fPIC", "-shared", "-fno-omit-frame-pointer",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Xarch_host", "-g",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
]


def build_host_sanitized(out_dir):
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, "libnufold_hostsan.so")
    cmd = [HIPCC, *SANITIZE_FLAGS, "-o", lib, *[os.path.join(CSRC, s) for s in SOURCES]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building the host-sanitized library")
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
