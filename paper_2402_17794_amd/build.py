"""Build librsvd.so (gfx950) in the package directory with hipcc.

    python -m paper_2402_17794_amd.build        # or build() from Python

Every source in csrc/ is compiled to an object in _build/ (in parallel), then
linked into paper_2402_17794_amd/librsvd.so.  The library links only the HIP
runtime; it has no dependency on torch.
"""

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librsvd.so")
ARCH = os.environ.get("RSVD_OFFLOAD_ARCH", "gfx950")

SOURCES = ["gemm.hip", "gemm_lp.hip", "orth.hip", "svd.hip", "single_pass.hip", "rsvd.cpp", "server.cpp"]

COMMON_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # Never emit packed FP32 instructions (v_pk_*_f32).
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"]
    remarks = ["-Rpass-analysis=kernel-resource-usage"] if src.endswith(".hip") else []
    cmd = [_hipcc(), *lang, *COMMON_FLAGS, *remarks, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def _spills(remarks):
    """Kernels whose registers spill to scratch memory, from the compiler's
    kernel-resource-usage remarks: {kernel: scratch bytes per lane}."""
    out, name = {}, None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name and int(m.group(1)) > 0:
            out[name] = int(m.group(1))
    return out


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    spills = {}
    for _, err in results:
        spills.update(_spills(err))
        if verbose:
            msgs = "\n".join(x for x in err.splitlines()
                             if x.strip() and "remark:" not in x and not re.match(r"\s*\d*\s*\|", x))
            if msgs:
                print(msgs, file=sys.stderr)
    with open(os.path.join(BUILD, "spills.txt"), "w") as f:
        for k, v in sorted(spills.items()):
            f.write(f"{k} {v}\n")
    if spills:
        # Register spills turn the single-workgroup kernels into scratch-bound code.
        print("warning: kernels spill registers to scratch: " + ", ".join(f"{k} ({v} B/lane)" for k, v in spills.items()),
              file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *[o for o, _ in results]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
