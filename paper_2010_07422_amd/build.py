"""Build libircur.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: python -m paper_2010_07422_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libircur.so")
SOURCES = ["ircur_kernels.hip", "ircur_pass16.hip", "ircur_svd.hip", "ircur_csvd.hip", "ircur_export.hip", "ircur_alg2.hip", "ircur_unrolled.hip", "ircur_unrolled_api.hip",
           "ircur_capi.hip"]
ARCH = os.environ.get("IRCUR_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",            # every fused multiply-add is written out
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{os.path.join(ROOT, 'include')}",
]


# Per-source device flags: the one-launch SVD keeps its matrix-core
# accumulators in ordinary vector registers (no copies to and from the
# accumulation registers around every product in its loops).
SRC_FLAGS = {
    "ircur_csvd.hip": ["-Xarch_device", "-mllvm=-amdgpu-mfma-vgpr-form"],
    "ircur_pass16.hip": ["-Xarch_device", "-mllvm=-amdgpu-mfma-vgpr-form"],
}


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "warning generated" not in l
                    and "warnings generated" not in l)
    if res.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + out)
    return out


def build(verbose: bool = False, jobs: int = 3, out: str | None = None,
          defines: tuple = ()) -> str:
    """Compile every HIP source to an object and link libircur.so (or `out`)."""
    from concurrent.futures import ThreadPoolExecutor
    lib_path = out or LIB
    objdir = os.path.join(PKG, "_build" if not defines else "_build_" + "_".join(defines))
    os.makedirs(objdir, exist_ok=True)

    def comp(src):
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, *SRC_FLAGS.get(src, ()), *("-D" + d for d in defines), "-c", os.path.join(CSRC, src),
               "-o", obj]
        out = _run(cmd)
        if verbose and out.strip():
            print(out)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(comp, SOURCES))
    tmp = lib_path + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
