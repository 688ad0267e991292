"""Measured HBM traffic of the K-product kernels, for the roofline report.

The figure comes from two rocprofv3 counter runs of ``python bench.py --probe``
-- one with FETCH_SIZE, one with WRITE_SIZE (both in KiB per dispatch) --
each scaled by what the same counter reads for the plain 256 MiB device copy
the probe makes after its solve (the counters do not cover every memory
channel alike, so the copy of known size calibrates them).  ``summarize``
writes ``profiles/traffic_<workload>.json`` with the bytes per launch of each
kernel kind and a hash of the kernel sources; ``load`` returns a kind's bytes
only while the sources still hash the same, else None.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/regpass.hip", "csrc/sepconv.hip", "csrc/kernels.hip", "csrc/fcrkpm.hip",
           "csrc/fcrkpm_impl.hpp", "csrc/fft_core.hpp"]
COPY_BYTES = 256 << 20

# demangled kernel name -> the kind name the library's sampler reports; the
# register passes are templates on the real type (", float>" / ", double>"
# at the end; older builds had no type argument)
_PASS = r"k_rpass<[^,]+(?:, \d+>)?, [^,]+, \d, "
_T32 = r"(, (true|false))?(, float)?>"
_T64 = r", (true|false), double>"
_KINDS = [
    (r"k_rmid2?<", "sep_mid_k_f32"),
    (r"k_smid<.*, float>", "sep_mid_k_f32"),
    (r"k_smid<.*, double>", "sep_mid_k_f64"),
    (_PASS + r"true, true, false, 1, 0" + _T32, "sep_part1_x_f32"),
    (_PASS + r"false, false, false, 1, 1" + _T32, "sep_part1_y_f32"),
    (_PASS + r"false, false, false, 2, 1" + _T32, "sep_part2_y_f32"),
    (_PASS + r"true, false, true, 2, 0" + _T32, "sep_part2_x_f32"),
    (_PASS + r"true, true, false, 1, 0" + _T64, "sep_part1_x_f64"),
    (_PASS + r"false, false, false, 1, 1" + _T64, "sep_part1_y_f64"),
    (_PASS + r"false, false, false, 2, 1" + _T64, "sep_part2_y_f64"),
    (_PASS + r"true, false, true, 2, 0" + _T64, "sep_part2_x_f64"),
]

_LAYOUT = r"(G16L?|G32|G8<\d+>|GPQ<\d+, \d+>)"


def _layout_index(lay):
    """Layout 1 is the 16-lane layout of 128-point lines, the 32-lane one of
    256-point lines and the 8-lane P x Q layouts of 80 and 96 points."""
    if lay.startswith(("G16", "G32")):
        return 1
    m = re.match(r"GPQ<\d+, (\d+)>", lay)
    return 1 if m and m.group(1) == "8" and lay not in ("GPQ<4, 8>", "GPQ<6, 8>") else 0


def _variant(name):
    """Register-path variant of a kernel name: layout + 2 (tiles - 1).  The pass
    kernels carry the basis after the layout; the middle passes do not, and the
    line-constant middle pass has one tile per workgroup in every variant."""
    m = re.search(r"k_rpass<[^<>]*?" + _LAYOUT + r", [^,]+, (\d)", name) or \
        re.search(r"k_rmid2?<[^<>]*?" + _LAYOUT + r", (\d)", name)
    if m:
        return _layout_index(m.group(1)) + 2 * (int(m.group(2)) - 1)
    m = re.search(r"k_smid<[^<>]*?" + _LAYOUT, name)
    if m:
        return _layout_index(m.group(1))
    return None


def source_hash() -> str:
    h = hashlib.sha256()
    for s in SOURCES:
        with open(os.path.join(HERE, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _per_kernel(path, counter):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def _calibration(vals):
    """KiB the counter reads for the 256 MiB copy (the largest copy dispatch)."""
    best = 0.0
    for name, v in vals.items():
        if "copyBuffer" in name or "direct_copy" in name:
            best = max(best, max(v))
    if best <= 0:
        raise ValueError("no calibration copy in the counter run")
    return best


def summarize(fetch_csv, write_csv, out_json, workload, command):
    fv = _per_kernel(fetch_csv, "FETCH_SIZE")
    wv = _per_kernel(write_csv, "WRITE_SIZE")
    cf = COPY_BYTES / (1024.0 * _calibration(fv))
    cw = COPY_BYTES / (1024.0 * _calibration(wv))
    kinds = {}
    for name in fv:
        for pat, kind in _KINDS:
            if re.search(pat, name) and name in wv:
                f = sum(fv[name]) / len(fv[name]) * 1024.0 * cf
                w = sum(wv[name]) / len(wv[name]) * 1024.0 * cw
                if kind in kinds and kinds[kind]["dispatches"] >= len(fv[name]):
                    continue  # keep the layout the solve ran (most dispatches)
                kinds[kind] = {"kernel": re.sub(r"\(.*", "", name.replace("(anonymous namespace)::", "")),
                               "layout": _variant(name),
                               "dispatches": len(fv[name]), "fetch_bytes": f, "write_bytes": w,
                               "bytes_per_launch": f + w}
    out = {"workload": workload, "source_hash": source_hash(), "copy_bytes": COPY_BYTES,
           "fetch_scale": cf, "write_scale": cw, "command": command, "kinds": kinds}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    return out


def load(workload, kind, layout=None, path=None):
    """Measured bytes per launch of `kind`, or None if not measured for the
    current kernel sources (and, if given, the same register variant)."""
    if path is None:
        path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kinds", {}).get(kind)
    if k is None:
        return None
    if layout is not None:
        # the line-constant middle pass has one tile per workgroup in every variant
        lay = layout & 1 if "smid" in k.get("kernel", "") else layout
        if k.get("layout") != lay:
            return None
    return k["bytes_per_launch"]


if __name__ == "__main__":
    # python -m paper_2403_19854_amd.traffic FETCH.csv WRITE.csv OUT.json WORKLOAD "COMMAND"
    print(json.dumps(summarize(*sys.argv[1:6]), indent=1))
