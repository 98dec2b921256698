"""Workload and summary for the rocprofv3 HBM-traffic counters of the headline step.

Counters are taken in two runs of their own (FETCH_SIZE, then WRITE_SIZE: the two do
not fit one pass):

  rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o run --output-format csv -- \\
      python3 paper_2210_06232_amd/profiling.py run
  rocprofv3 --pmc WRITE_SIZE -d OUT/write -o run --output-format csv -- \\
      python3 paper_2210_06232_amd/profiling.py run
  python3 paper_2210_06232_amd/profiling.py summarize OUT/fetch OUT/write

(`run --preset i [--inputs-cache DIR]` takes a named preset of workload.py instead, and
`summarize ... OUT.json --note TEXT` writes elsewhere.)

Shader-sequencer counters (instruction mix, issue and wait shares, LDS bank conflicts)
take one run per group of SQ_PASSES, then `sq DIR1 DIR2 --out FILE.md`.

`run` does a few FP64 and FP32 steps of the headline workload, then three plain device
copies of a known size (the copy kernel calibrates the counters: its true traffic is
the buffer size read plus the buffer size written).  `summarize` writes
profiles/traffic_256cubed.json: per kernel and precision, HBM bytes per launch from
the counters scaled by the copy's factor, stamped with the hash of the kernel sources
they were taken on.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 6 * 256 ** 3 * 8  # one FP64 state of the headline grid
OUT_JSON = os.path.join(ROOT, "profiles", "traffic_256cubed.json")


# the sources that define the step's kernels and their launch shapes
KERNEL_SOURCES = ("fft_core.h", "kernels.h", "small_plane.h", "passes.h", "passes_impl.h", "passes_f64.hip",
                  "passes_f32.hip", "passes_c2c_f64.hip", "passes_c2c_f32.hip")


def code_text(src: str) -> str:
    """The source with comments removed and whitespace runs collapsed: what the hash of
    the kernel sources covers, so that editing a comment does not mark the counters
    taken on the same code as stale."""
    out, i, n = [], 0, len(src)
    while i < n:
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif src[i] == '"':  # string literal (asm templates): copied whole
            j = i + 1
            while j < n and src[j] != '"':
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(src[i])
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2210_06232_amd", "csrc")
    from paper_2210_06232_amd.build import FILE_FLAGS  # per-source compiler flags change the code too
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode() + code_text(f.read()).encode())
        h.update(" ".join(FILE_FLAGS.get(name, [])).encode())
    return h.hexdigest()[:16]


def run(steps: int = 3, preset=None, cache=None):
    """A few steps of the headline workload in both precisions (or of a named preset in
    its own precisions), then the calibration copies."""
    import torch
    from paper_2210_06232_amd import eifp
    from paper_2210_06232_amd import workload
    if preset is None:
        cfg, precs = workload.HEADLINE, ("fp64", "fp32")
        H, E = workload.headline_inputs()
    else:
        cfg = workload.PRESETS[preset]
        precs = cfg["precs"]
        H, E = workload.preset_inputs(cfg, lambda m: print("[profiling]", m, flush=True), cache=cache)
    for prec in precs:
        with eifp.Solver(H, E, cfg["domain"], cfg["mu"], cfg["eps"], prec) as s:
            s.step(cfg["tau"], steps)
            s.sync()
        print(f"[profiling] {prec}: {steps} steps", flush=True)
    del H, E
    x = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("[profiling] copies done", flush=True)


def _rows(d: str, counter: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    yield r["Kernel_Name"], int(r["Dispatch_Id"]), float(r["Counter_Value"])


def _per_kernel(rows):
    """{(prec, name): [KiB per dispatch]} for the library kernels; copy dispatches apart."""
    out, copies = {}, []
    for name, _, v in rows:
        m = re.search(r"(k_[a-z0-9_]+)<(double|float)", name)
        if m:
            key = ("fp64" if m.group(2) == "double" else "fp32", m.group(1))
            out.setdefault(key, []).append(v)
        elif "copy" in name.lower():
            copies.append(v)
    return out, copies


def summarize(fetch_dir: str, write_dir: str, out_path: str = OUT_JSON, note=None):
    fk, fc = _per_kernel(_rows(fetch_dir, "FETCH_SIZE"))
    wk, wc = _per_kernel(_rows(write_dir, "WRITE_SIZE"))
    # the calibration copies are the largest copy dispatches
    big_f = [v for v in fc if v >= 0.5 * max(fc)]
    big_w = [v for v in wc if v >= 0.5 * max(wc)]
    f_kib, w_kib = sum(big_f) / len(big_f), sum(big_w) / len(big_w)
    ff, fw = COPY_BYTES / (f_kib * 1024.0), COPY_BYTES / (w_kib * 1024.0)
    kernels = {}
    for key in sorted(set(fk) | set(wk)):
        prec, name = key
        fv, wv = fk.get(key, [0.0]), wk.get(key, [0.0])
        f_mean, w_mean = sum(fv) / len(fv), sum(wv) / len(wv)
        kernels.setdefault(prec, {})[name] = {
            "dispatches": len(fv), "fetch_kib_raw": round(f_mean, 1), "write_kib_raw": round(w_mean, 1),
            "fetch_bytes": round(f_mean * 1024.0 * ff), "write_bytes": round(w_mean * 1024.0 * fw)}
    rec = {"source_hash": kernel_source_hash(), "copy_bytes": COPY_BYTES,
           "copy_fetch_kib_raw": round(f_kib, 1), "copy_write_kib_raw": round(w_kib, 1),
           "factor_fetch": ff, "factor_write": fw, "kernels": kernels,
           "note": note or "bytes per launch; one launch of a pass covers all six components of the 256^3 state"}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


# Shader-sequencer counters of the step's kernels, one rocprofv3 pass per group (a pass
# holds at most 8 SQ counters).
SQ_PASSES = (
    "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VMEM "
    "SQ_WAIT_INST_ANY SQ_WAIT_ANY",
    "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SALU SQ_LDS_BANK_CONFLICT "
    "SQ_WAIT_INST_LDS",
)
LDS_PER_CU = 160 * 1024


def _waves_per_simd(wg: int, vgpr: int, agpr: int, lds: int) -> int:
    """Resident waves per SIMD from the register and LDS footprint (512 registers per
    lane per SIMD, VGPRs and AGPRs allocated together in blocks of 8; 160 KB of LDS per
    CU; a workgroup's waves spread over the CU's 4 SIMDs)."""
    regs = -(-(vgpr + agpr) // 8) * 8
    by_regs = 512 // max(regs, 8)
    wg_waves = -(-wg // 64)
    by_lds = (LDS_PER_CU // lds) * wg_waves / 4 if lds else 8
    return int(min(8, by_regs, by_lds))


def sq_summary(dirs, out_path: str, title: str):
    """Per kernel (name and template arguments) and precision: the SQ counters averaged
    over its dispatches, per wave where they count instructions, with the footprint the
    trace records (VGPRs, AGPRs, LDS) and the waves per SIMD it allows."""
    vals, meta = {}, {}
    for d in dirs:
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(fn) as f:
                for r in csv.DictReader(f):
                    name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("eifp::", "")
                    if not name.startswith("k_") or name.startswith("k_twiddles"):
                        continue
                    vals.setdefault(name, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                    meta[name] = (int(r["Workgroup_Size"]), int(r["VGPR_Count"]), int(r["Accum_VGPR_Count"]),
                                  int(r["LDS_Block_Size"]))
    avg = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in vals.items()}
    lines = [f"# {title}", "",
             "Counters averaged over each kernel's dispatches; per-wave figures divide by SQ_WAVES.",
             "Cycle counters (SQ_*_CYCLES, SQ_ACTIVE_INST_*, SQ_WAIT_*) are in the sequencer's own",
             "units; only their ratios are used: issue and wait shares of the waves' resident time",
             "(SQ_WAVE_CYCLES).", "",
             "| Kernel | WG | VGPR+AGPR | LDS (B) | waves/SIMD | waves | VALU/wave | LDS/wave | VMEM rd+wr/wave "
             "| VALU share | LDS share | VMEM share | dependency wait | any wait | bank-conflict / LDS-active |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    rec = {}
    for k in sorted(avg):
        a = avg[k]
        wg, vg, ag, lds = meta[k]
        w = a.get("SQ_WAVES", 0.0)
        wc = a.get("SQ_WAVE_CYCLES", 0.0)
        per = lambda c: a[c] / w if w and c in a else None
        share = lambda c: a[c] / wc if wc and c in a else None
        vm = (per("SQ_INSTS_VMEM_RD") or 0.0) + (per("SQ_INSTS_VMEM_WR") or 0.0)
        bc = a["SQ_LDS_BANK_CONFLICT"] / a["SQ_ACTIVE_INST_LDS"] if a.get("SQ_ACTIVE_INST_LDS") and \
            "SQ_LDS_BANK_CONFLICT" in a else None
        row = {"workgroup": wg, "vgpr": vg, "agpr": ag, "lds_bytes": lds,
               "waves_per_simd": _waves_per_simd(wg, vg, ag, lds), "waves": w,
               "valu_per_wave": per("SQ_INSTS_VALU"), "lds_per_wave": per("SQ_INSTS_LDS"), "vmem_per_wave": vm,
               "valu_share": share("SQ_ACTIVE_INST_VALU"), "lds_share": share("SQ_ACTIVE_INST_LDS"),
               "vmem_share": share("SQ_ACTIVE_INST_VMEM"), "dep_wait_share": share("SQ_WAIT_INST_ANY"),
               "any_wait_share": share("SQ_WAIT_ANY"), "bank_conflict_per_lds_active": bc, "raw": a}
        rec[k] = row
        f = lambda x, p=3: "–" if x is None else (f"{x:.{p}f}" if isinstance(x, float) else str(x))
        lines.append(f"| `{k}` | {wg} | {vg}+{ag} | {lds} | {row['waves_per_simd']} | {w:.0f} | "
                     f"{f(row['valu_per_wave'], 0)} | {f(row['lds_per_wave'], 0)} | {f(vm, 0)} | "
                     f"{f(row['valu_share'])} | {f(row['lds_share'])} | {f(row['vmem_share'])} | "
                     f"{f(row['dep_wait_share'])} | {f(row['any_wait_share'])} | {f(bc)} |")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.splitext(out_path)[0] + ".json", "w") as f:
        json.dump({"source_hash": kernel_source_hash(), "kernels": rec}, f, indent=1)
    print("\n".join(lines))


def main(argv):
    import argparse
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("steps", type=int, nargs="?", default=3)
    r.add_argument("--preset", type=int, default=None, help="a named preset instead of the headline workload")
    r.add_argument("--inputs-cache", default=None)
    m = sub.add_parser("summarize")
    m.add_argument("fetch_dir")
    m.add_argument("write_dir")
    m.add_argument("out", nargs="?", default=OUT_JSON)
    m.add_argument("--note", default=None)
    q = sub.add_parser("sq", help="summarise SQ counter runs (one directory per pass of SQ_PASSES)")
    q.add_argument("dirs", nargs="+")
    q.add_argument("--out", required=True)
    q.add_argument("--title", default="SQ counters of the step's kernels")
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run(a.steps, a.preset, a.inputs_cache)
    elif a.cmd == "sq":
        sq_summary(a.dirs, a.out, a.title)
    else:
        summarize(a.fetch_dir, a.write_dir, a.out, a.note)


if __name__ == "__main__":
    main(sys.argv[1:])
