"""Build libgm.so for gfx950 with hipcc (in-tree, no JIT cache).

python -m paper_2602_13198_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "csrc", "gm_api.hip")
OUT_DIR = os.path.join(_HERE, "_lib")
OUT = os.path.join(OUT_DIR, "libgm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep hand-free of packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    # fuse a*b+c only within one source expression, so that every compiled
    # variant of a kernel rounds the same expression the same way
    "-ffp-contract=on",
    # uniform-address LDS atomics (tallies, ledgers) issued per lane: the
    # default rewrite into a per-lane readlane loop costs more VALU than the
    # LDS unit's own serialisation of the conflicting lanes
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


def resources() -> str:
    """Per-kernel register, scratch, LDS and occupancy figures as the
    compiler reports them for this build (-Rpass-analysis=kernel-resource-usage),
    as a text table.  Dynamic LDS (tallies, event staging) is set per launch
    and not part of these figures."""
    import re
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        cmd = [HIPCC] + [f for f in FLAGS if f not in ("-shared", "-fPIC")] + [
            "-c", "-Rpass-analysis=kernel-resource-usage", "-o", os.path.join(d, "gm.o"), SRC]
        r = subprocess.run(cmd, capture_output=True, text=True, check=True)
    rows, cur = [], None
    for line in r.stderr.splitlines():
        m = re.search(r"remark:\s+(Function Name|VGPRs Spill|VGPRs|AGPRs|TotalSGPRs|ScratchSize \[bytes/lane\]|"
                      r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]): (\S+)", line)
        if not m:
            continue
        k, v = m.group(1), m.group(2)
        if k == "Function Name":
            cur = {"name": v}
            rows.append(cur)
        elif cur is not None:
            cur[{"VGPRs Spill": "Spill", "TotalSGPRs": "SGPRs"}.get(k, k.split(" ")[0])] = v
    keep = [x for x in rows if "_ZN2gm" in x["name"] and "kernel" in x["name"]]
    out = ["# kernel resources of libgm.so for gfx950 (compiler report)",
           "# command: python -m paper_2602_13198_amd.build --resources",
           "# kernel | VGPRs | AGPRs | SGPRs | VGPR spills | scratch B/lane | static LDS B/block | occupancy waves/SIMD"]
    for x in keep:
        out.append("%s | %s | %s | %s | %s | %s | %s | %s" % (
            x["name"], x.get("VGPRs", "?"), x.get("AGPRs", "?"), x.get("SGPRs", "?"), x.get("Spill", "?"),
            x.get("ScratchSize", "?"), x.get("LDS", "?"), x.get("Occupancy", "?")))
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    if "--resources" in sys.argv:
        sys.stdout.write(resources())
    else:
        print(build(verbose="-v" in sys.argv))
