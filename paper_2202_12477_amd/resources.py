"""Per-degree register, LDS and occupancy table of the operator kernels.

Compiles the operator's translation units (device code only, gfx950) with the
compiler's kernel-resource-usage remarks and prints, for every degree N,
precision and tile schedule, the single-problem operator kernel's VGPRs,
spilled VGPRs, scratch, LDS per workgroup, workgroup shape, idle lanes and the
waves per SIMD the compiler reports (the analogue of the occupancy table the
paper gives for its high-degree kernels).  Default schedules are marked *.

  python -m paper_2202_12477_amd.resources [--cg] [--markdown]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import subprocess

from paper_2202_12477_amd import build as hbuild

UNITS = ["ax_n1_5.hip", "ax_n6_10.hip", "ax_n11_15.hip"]
FIELDS = {"VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch", "Occupancy [waves/SIMD]": "occ",
          "VGPRs Spill": "vspill", "SGPRs Spill": "sspill", "LDS Size [bytes/block]": "lds", "TotalSGPRs": "sgpr"}
# the default schedule table of csrc/ax.hip (FP64 row, FP32 row), read from the source
_SCHED_RE = re.compile(r"\{([0-9, ]+)\},\s*//\s*(FP64|FP32)")


def default_schedules():
    src = open(os.path.join(hbuild.CSRC, "ax.hip")).read()
    out = {}
    for vals, prec in _SCHED_RE.findall(src):
        out[prec] = [int(v) for v in vals.split(",")]
    return out


def remarks(unit: str) -> str:
    src = os.path.join(hbuild.CSRC, unit)
    cmd = [hbuild.HIPCC, *hbuild.FLAGS, "-x", "hip", "--cuda-device-only", "-c", src, "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-4000:])
    return r.stderr


def parse(text: str):
    kernels, cur = [], None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = {"mangled": m.group(1)}
            kernels.append(cur)
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+(?:\[[^\]]*\])?): (\S+)", line)
        if m and cur is not None and m.group(1).strip() in FIELDS:
            v = m.group(2)
            cur[FIELDS[m.group(1).strip()]] = int(v) if v.lstrip("-").isdigit() else v
    names = subprocess.run(["c++filt"], input="\n".join(k["mangled"] for k in kernels), capture_output=True,
                           text=True).stdout.splitlines()
    for k, n in zip(kernels, names):
        k["name"] = n
    return kernels


def shape(N: int, sched: int):
    np2 = (N + 1) ** 2
    target = 64 if (sched & 2) and np2 <= 64 else 256
    epb = max(target // np2, 1)
    threads = (epb * np2 + 63) // 64 * 64
    return epb, threads, 1.0 - epb * np2 / threads


def table(cg: bool = False):
    with cf.ThreadPoolExecutor(len(UNITS)) as ex:
        texts = list(ex.map(remarks, UNITS))
    rows = []
    pat = re.compile(r"hb::ax_kernel<(\d+), (true|false), (double|float), (\d+), false>")
    for k in (k for t in texts for k in parse(t)):
        m = pat.search(k["name"])
        if not m or (m.group(2) == "true") != cg:
            continue
        N, prec, sched = int(m.group(1)), "FP64" if m.group(3) == "double" else "FP32", int(m.group(4))
        epb, threads, idle = shape(N, sched)
        rows.append(dict(N=N, prec=prec, sched=sched, epb=epb, threads=threads, idle=idle, **{
            f: k.get(f) for f in FIELDS.values()}))
    rows.sort(key=lambda r: (r["prec"] != "FP64", r["N"], r["sched"]))
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--cg", action="store_true", help="the CG form of the kernel (fused p.Ap partials)")
    ap.add_argument("--markdown", action="store_true")
    a = ap.parse_args()
    dflt = default_schedules()
    rows = table(a.cg)
    hdr = ["prec", "N", "sched", "elem/WG", "threads", "idle lanes", "VGPR", "AGPR", "VGPR spill", "scratch B/lane",
           "LDS B/WG", "waves/SIMD"]
    if a.markdown:
        print("| " + " | ".join(hdr) + " |")
        print("|" + "---|" * len(hdr))
    else:
        print("  ".join(hdr))
    for r in rows:
        star = "*" if dflt.get(r["prec"], [0] * 16)[r["N"]] == r["sched"] else ""
        vals = [r["prec"], r["N"], f"{r['sched']}{star}", r["epb"], r["threads"], f"{100 * r['idle']:.0f}%", r["vgpr"],
                r["agpr"], r["vspill"], r["scratch"], r["lds"], r["occ"]]
        print(("| " + " | ".join(map(str, vals)) + " |") if a.markdown else "  ".join(map(str, vals)))


if __name__ == "__main__":
    main()
