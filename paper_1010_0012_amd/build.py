"""Build libbp_hip.so (HIP, gfx950) in-tree.

Every translation unit under csrc/ is compiled with hipcc for gfx950 in
parallel, then linked into paper_1010_0012_amd/libbp_hip.so.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbp_hip.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # every fused multiply-add in the kernels is an explicit fmaf: no implicit
    # contraction, so two kernels running the same source round the same way
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    noisy = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if noisy:
        sys.stderr.write("\n".join(noisy) + "\n")
    return obj


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), max(1, min(8, (os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


# The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer,
# with the BP_DEBUG checks of the host code: host-side compilation only (no
# device code), linked with the host check program tests/host/host_runtime.cpp
# into _build/san/host_runtime.  The sanitizer flags apply to the host pass
# only (-Xarch_host).
SAN_FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--cuda-host-only", "-x", "hip", "-DBP_DEBUG",
             "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
SAN_DIR = os.path.join(BUILD, "san")
SAN_PROGRAM = os.path.join(SAN_DIR, "host_runtime")
SAN_HARNESS = os.path.join(ROOT, "tests", "host", "host_runtime.cpp")


def _compile_san(src):
    obj = os.path.join(SAN_DIR, os.path.basename(src).rsplit(".", 1)[0] + ".o")
    cmd = [HIPCC, *SAN_FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _device_bundle_placeholders(objs):
    """Host-only objects still name the device-code bundle of their
    translation unit (__hip_fatbin_<id>), which only a device compilation
    defines.  The check program never launches a kernel and runs only where
    there is no GPU, so zero-filled placeholders satisfy the references."""
    nm = shutil.which("nm") or "/opt/rocm/lib/llvm/bin/llvm-nm"
    names = set()
    for o in objs:
        out = subprocess.run([nm, o], capture_output=True, text=True, check=True).stdout
        names.update(ln.split()[-1] for ln in out.splitlines() if ln.split()[-2:-1] == ["U"]
                     and ln.split()[-1].startswith("__hip_fatbin_"))
    src = os.path.join(SAN_DIR, "device_bundle_placeholders.cpp")
    with open(src, "w") as f:
        for n in sorted(names):
            f.write(f'extern "C" __attribute__((aligned(4096))) const char {n}[64] = {{0}};\n')
    obj = src[:-4] + ".o"
    subprocess.run([HIPCC, "-c", src, "-o", obj], capture_output=True, text=True, check=True)
    return obj


def build_sanitized():
    """Build _build/san/host_runtime (see above) and return its path."""
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = sources() + [SAN_HARNESS]
    with cf.ThreadPoolExecutor(min(len(srcs), 8)) as ex:
        objs = list(ex.map(_compile_san, srcs))
    objs.append(_device_bundle_placeholders(objs))
    cmd = [HIPCC, "-Xarch_host", "-fsanitize=address,undefined", "-o", SAN_PROGRAM, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return SAN_PROGRAM


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "sanitized":
        print(build_sanitized())
    else:
        build()
