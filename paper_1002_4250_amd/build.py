"""Build libtsqr.so for gfx950 from the sources in csrc/.

One translation unit per kernel instantiation listed in
``csrc/tsqr_instances.h`` is compiled with hipcc in parallel, then linked with
the C-ABI layer into ``paper_1002_4250_amd/libtsqr.so`` (in-tree, so that it
travels with the repository).  ``python -m paper_1002_4250_amd.build`` builds
from the command line.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libtsqr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ARCH = "gfx950"
# packed FP32 instructions are kept out of every kernel
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++20", "-fPIC", "-I" + INCLUDE, "-I" + CSRC] + DEVICE_FLAGS


def instances():
    """(kind, defines) for every translation unit, parsed from tsqr_instances.h."""
    text = open(os.path.join(CSRC, "tsqr_instances.h")).read()
    leaf_block = re.search(r"#define TSQR_LEAF_INSTANCES\(X\)(.*?)\n\n", text, re.S).group(1)
    op_block = re.search(r"#define TSQR_OP_INSTANCES\(O\)(.*?)\n\n", text, re.S).group(1)
    qr_block = re.search(r"#define TSQR_QR_INSTANCES\(Q\)(.*?)\n\n", text, re.S).group(1)
    units = [("common", ["-DTSQR_INST_COMMON"])]
    for tag, nc, rpl in re.findall(r"X\((\w+),\s*(\d+),\s*(\d+)\)", leaf_block):
        units.append((f"leaf_{tag}_{nc}_{rpl}",
                      ["-DTSQR_INST_LEAF", f"-DTSQR_INST_TAG={tag}", f"-DTSQR_INST_NC={nc}",
                       f"-DTSQR_INST_RPL={rpl}"]))
    for tag, nc in re.findall(r"O\((\w+),\s*(\d+)\)", op_block):
        units.append((f"op_{tag}_{nc}", ["-DTSQR_INST_OP", f"-DTSQR_INST_TAG={tag}", f"-DTSQR_INST_NC={nc}"]))
    for tag, nc, rpl in re.findall(r"Q\((\w+),\s*(\d+),\s*(\d+)\)", qr_block):
        units.append((f"qr_{tag}_{nc}_{rpl}",
                      ["-DTSQR_INST_QR", f"-DTSQR_INST_TAG={tag}", f"-DTSQR_INST_NC={nc}",
                       f"-DTSQR_INST_RPL={rpl}"]))
    return units


KERNEL_DEPS = ["tsqr_inst.hip", "tsqr_device.h", "tsqr_mixed.h", "tsqr_q.h", "tsqr_internal.h", "tsqr_instances.h",
               "tsqr_mlp.h"]
API_DEPS = ["tsqr_api.cpp", "tsqr_internal.h", "tsqr_instances.h", "tsqr_mixed.h", "tsqr_device.h"]


def _digest(names):
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + f.read())
    with open(os.path.join(INCLUDE, "tsqr.h"), "rb") as f:
        h.update(f.read())
    # the compiler flags, without the include paths: the digest must not depend
    # on where the repository sits
    h.update(" ".join(f for f in COMMON if not f.startswith("-I")).encode())
    return h.hexdigest()[:16]


def _compile(args):
    out, cmd = args
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (out, " ".join(cmd), r.stderr[-4000:]))
    return out


def build(force: bool = True, jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every instantiation and link libtsqr.so.  With force=False,
    objects whose source digest is unchanged are reused."""
    os.makedirs(BUILD, exist_ok=True)
    kdig, adig = _digest(KERNEL_DEPS), _digest(API_DEPS)
    tasks = []
    objs = []
    for name, defs in instances():
        obj = os.path.join(BUILD, f"{name}.{kdig}.o")
        objs.append(obj)
        if force or not os.path.exists(obj):
            src = os.path.join(CSRC, "tsqr_inst.hip")
            tasks.append((obj, [HIPCC] + COMMON + defs + ["-c", src, "-o", obj + ".tmp"]))
    api_obj = os.path.join(BUILD, f"api.{adig}.o")
    if force or not os.path.exists(api_obj):
        tasks.append((api_obj, [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, "tsqr_api.cpp"),
                                                   "-o", api_obj + ".tmp"]))
    objs.append(api_obj)
    jobs = jobs or min(16, os.cpu_count() or 4)
    # the largest units first so the pool finishes evenly
    tasks.sort(key=lambda t: (0 if ("leaf_" in t[0] or "qr_" in t[0]) else 1, t[0]))
    with cf.ThreadPoolExecutor(max_workers=jobs) as pool:
        for done in pool.map(_compile, tasks):
            os.replace(done + ".tmp", done)
            if verbose:
                print("built", os.path.basename(done), flush=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    _compile((tmp, [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs))
    os.replace(tmp, LIB)
    # drop objects of older source versions
    keep = set(os.path.basename(o) for o in objs)
    for name in os.listdir(BUILD):
        if name.endswith(".o") and name not in keep:
            os.remove(os.path.join(BUILD, name))
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)
    if os.path.exists(LIB):
        os.remove(LIB)


if __name__ == "__main__":
    force = "--incremental" not in sys.argv
    print(build(force=force, verbose=True))
