"""Build librbm.so (the gfx950 HIP library behind include/rbm.h) in-tree with hipcc, and
abi_check: a program that walks the C ABI (tests/abi_check.cpp) linked against the same
kernels with the library's host code (rbm_api.cpp, rbm_static.cpp) rebuilt under
AddressSanitizer and UndefinedBehaviorSanitizer.  The sanitizers apply to host code only
(each flag behind -Xarch_host); the gfx950 code objects are the ordinary ones.

    python -m paper_1606_07428_amd.build        (or __graft_entry__.build())
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librbm.so")
ABI_CHECK = os.path.join(HERE, "abi_check")
ABI_CHECK_SRC = os.path.join(ROOT, "tests", "abi_check.cpp")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 VALU ops are disabled for every HIP translation unit
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]


# host-side sanitizers for the ABI check; never applied to device code
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src, sanitize=False):
    sub = os.path.join(BUILD, "san") if sanitize else BUILD
    os.makedirs(sub, exist_ok=True)
    obj = os.path.join(sub, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + (SAN + ["-g"] if sanitize else []) + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    kern = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    host = sorted(glob.glob(os.path.join(CSRC, "*.cpp")))
    srcs = kern + host
    jobs = [(x, False) for x in srcs] + [(x, True) for x in host + [ABI_CHECK_SRC]]
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        built = list(ex.map(lambda j: _compile(*j), jobs))
    objs, san_objs = built[:len(srcs)], built[len(srcs):]
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    tmp = ABI_CHECK + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}"] + SAN + ["-o", tmp] + objs[:len(kern)] + san_objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link of abi_check failed:\n{r.stderr}")
    os.replace(tmp, ABI_CHECK)
    if verbose:
        print(f"built {OUT} and {ABI_CHECK}")
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
