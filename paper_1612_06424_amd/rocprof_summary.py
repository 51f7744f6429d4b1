"""Condense rocprofv3 output of bench.py into the short text kept under profiles/.

    python -m paper_1612_06424_amd.rocprof_summary DIR [--keep-raw]

profile_bench.sh beside this file runs the passes and then this module.  DIR holds one
rocprofv3 output directory per pass (csv format):
  trace/       --kernel-trace --stats of the bench
  fetch/       --pmc FETCH_SIZE  (stencil kernels: dslash and half-hop instances)
  write/       --pmc WRITE_SIZE  (stencil kernels)
  copy_fetch/  --pmc FETCH_SIZE  of bench.py --copy-calibration
  copy_write/  --pmc WRITE_SIZE  of bench.py --copy-calibration
  units/       (optional) --pmc of the vector-memory unit counters TA_TA_BUSY_sum,
               TA_ADDR_STALLED_BY_TC_CYCLES_sum, TCP_TCR_TCP_STALL_CYCLES_sum,
               TCP_PENDING_STALL_CYCLES_sum, TCP_TOTAL_CACHE_ACCESSES_sum, SQ_INSTS_VMEM_RD,
               GRBM_GUI_ACTIVE (stencil kernels)
and writes DIR/summary.md (per-kernel durations, HBM bytes per launch from
the counters scaled by the copy calibration) and DIR/stencil_traffic.json,
which bench.py reads to fill roofline.traffic while the stencil sources are
unchanged (same kernel_source_hash).  Raw csv files are deleted unless
--keep-raw (they are large).
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
# the sources that decide what the stencil kernels do and how they are launched
STENCIL_SOURCES = ["csrc/dd_dslash.h", "csrc/dd_eo.h", "csrc/dd_eo_lds.h", "csrc/dd_wilson.h", "csrc/dd_internal.h",
                   "csrc/dirac.hip", "csrc/evenodd.hip", "csrc/batched.hip", "csrc/tune.hip", "tune_cache_mi355x.txt"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in STENCIL_SOURCES:
        p = os.path.join(PKG, rel)
        h.update(rel.encode())
        if os.path.exists(p):
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def short_name(n: str) -> str:
    m = re.search(r"(k_\w+<[^()]*>|k_\w+|__amd_\w+)", n)
    return m.group(1) if m else n[:48]


def timing_name(k: str) -> str:
    """The library's HIP-event timing name of a kernel instance: the full stencil's timing name
    omits its last template argument (x hops through lane permutes or not), and with one column
    per thread the column count as well."""
    if not k.startswith("k_dslash<"):
        return k
    args = [a.strip() for a in k[len("k_dslash<"):-1].split(",")]
    if len(args) == 6:
        args = args[:5]
    if len(args) == 5 and args[4] == "1":
        args = args[:4]
    return "k_dslash<" + ", ".join(args) + ">"


HEADER = """# Stencil and solver kernels of the bench workload (64x32^3 lattice, its 16x32^3 slabs, 96 batched domains, 32x16^3 force domain)

Command (repository root, one MI355X): `bash paper_1612_06424_amd/profile_bench.sh OUT`, which runs,
with `DD_TUNE_CACHE` naming a copy of `paper_1612_06424_amd/tune_cache_mi355x.txt` (so that every pass
launches the same kernel instances), B = `bench.py --steps 1 --warmup 1 --no-cpu-baseline --parts
stencil,solve,fact,batched,force` and SEL = `--kernel-include-regex "dslash|eo_hop|eo_lds"`:

    cd /tmp && export TMPDIR=/tmp
    rocprofv3 --kernel-trace --stats -f csv -d OUT/trace -o run -- python3 B > OUT/trace.log
    rocprofv3 --pmc FETCH_SIZE -f csv -d OUT/copy_fetch -o run -- python3 bench.py --copy-calibration
    rocprofv3 --pmc WRITE_SIZE -f csv -d OUT/copy_write -o run -- python3 bench.py --copy-calibration
    rocprofv3 --pmc FETCH_SIZE SEL -f csv -d OUT/fetch -o run -- python3 B
    rocprofv3 --pmc WRITE_SIZE SEL -f csv -d OUT/write -o run -- python3 B
    rocprofv3 --pmc TA_TA_BUSY_sum TA_ADDR_STALLED_BY_TC_CYCLES_sum TCP_TCR_TCP_STALL_CYCLES_sum \\
        TCP_PENDING_STALL_CYCLES_sum TCP_TOTAL_CACHE_ACCESSES_sum SQ_INSTS_VMEM_RD GRBM_GUI_ACTIVE SEL \\
        -f csv -d OUT/units -o run -- python3 B
    python3 -m paper_1612_06424_amd.rocprof_summary OUT

Kernel names: `k_dslash<real, dagger, epilogue, workgroup size, columns per thread, x hops from
neighbouring lanes>` is the time-sweep stencil (its HIP-event name omits the last argument, and the
column count when it is 1) (epilogue 0 store, 1 <aux, D in>, 2 <D in, in> and |D in|^2, 3 residual,
4 |D in|^2, 5 kappa D_hop in); `k_eo_hop<real, dagger, epilogue, workgroup size, self, columns per
thread, two-row links>` is the even-odd half hop (`k_eo_hop_nt` the same with non-temporal output
stores; self = true: the second half of the Schur operator, or the source preparation /
reconstruction), `k_eo_lds<float, dagger, epilogue, self, L/2, non-temporal>` its LDS-tile form
(one slice per workgroup), `k_beo_hop<real, dagger, epilogue, self, columns per thread, two-row
links>` its multi-domain form in the batched solve.  The batched solve replays its inner
iterations as a HIP graph, whose launches the library's HIP-event timing does not see: for
`k_beo_hop` the HIP-event column averages the eager launches only, the rocprof column all of
them.  Algorithmic bytes per launch: V ((48 + e) ncol + 72) sizeof(real) for the full stencil,
(V/2) ((48 + e) ncol + 144) sizeof(real) for a half hop (e = 24 per extra field read: aux for
epilogues 1 and 3, the self field; 96 instead of 144 with two-row links), with ncol the live
columns.  `stencil_traffic.json` beside this file holds the per-launch HBM bytes that bench.py
reports as roofline.traffic while the hashed stencil sources are unchanged.

"""


def _rows(pattern):
    out = []
    for f in glob.glob(pattern, recursive=True):
        with open(f) as fh:
            out.extend(csv.DictReader(fh))
    return out


def counters(d):
    """{kernel: (dispatches, mean counter value per dispatch)} of one --pmc pass."""
    agg = collections.OrderedDict()
    for r in _rows(os.path.join(d, "**", "*counter_collection.csv")):
        k = short_name(r.get("Kernel_Name", "?"))
        a = agg.setdefault(k, [set(), 0.0])
        a[0].add(r.get("Dispatch_Id") or r.get("Correlation_Id"))
        a[1] += float(r.get("Counter_Value") or 0)
    return {k: (len(v[0]), v[1] / max(len(v[0]), 1)) for k, v in agg.items()}


def counters_by_name(d):
    """{kernel: {counter: mean value per dispatch}} of one --pmc pass with several counters."""
    agg = collections.OrderedDict()
    for r in _rows(os.path.join(d, "**", "*counter_collection.csv")):
        k = short_name(r.get("Kernel_Name", "?"))
        a = agg.setdefault(k, collections.OrderedDict())
        c = a.setdefault(r.get("Counter_Name", "?"), [set(), 0.0])
        c[0].add(r.get("Dispatch_Id") or r.get("Correlation_Id"))
        c[1] += float(r.get("Counter_Value") or 0)
    return {k: {c: v[1] / max(len(v[0]), 1) for c, v in cs.items()} | {"_n": max(len(v[0]) for v in cs.values())}
            for k, cs in agg.items()}


NCU = 256  # MI355X compute units: one texture-address unit (TA) and one vector L1 (TCP) each
NXCD = 8   # GRBM_GUI_ACTIVE reads the sum over the 8 XCDs (8 x the dispatch's clocks)


def units_table(d):
    """Busy and stall fractions of the vector-memory units per stencil kernel, as shares of
    NCU x the dispatch's GPU-active clocks (GRBM_GUI_ACTIVE / NXCD)."""
    u = counters_by_name(os.path.join(d, "units"))
    if not u:
        return []
    out = ["| kernel | launches (pmc) | clocks | TA busy | TA stalled by TC | TCP stalled by TCR | "
           "TCP pending stall | vector-memory reads / launch | L1 accesses / launch |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(u):
        c = u[k]
        cyc = c.get("GRBM_GUI_ACTIVE", 0.0) / NXCD
        if cyc <= 0:
            continue
        den = NCU * cyc

        def frac(name):
            return f"{c[name] / den:.2f}" if name in c else "-"

        out.append(f"| `{k}` | {c['_n']} | {cyc:.4g} | {frac('TA_TA_BUSY_sum')} | "
                   f"{frac('TA_ADDR_STALLED_BY_TC_CYCLES_sum')} | {frac('TCP_TCR_TCP_STALL_CYCLES_sum')} | "
                   f"{frac('TCP_PENDING_STALL_CYCLES_sum')} | {c.get('SQ_INSTS_VMEM_RD', 0):.4g} | "
                   f"{c.get('TCP_TOTAL_CACHE_ACCESSES_sum', 0):.4g} |")
    return out


def main(argv):
    d = argv[0]
    keep = "--keep-raw" in argv
    stats = _rows(os.path.join(d, "trace", "**", "*kernel_stats.csv"))
    cf, cw = counters(os.path.join(d, "copy_fetch")), counters(os.path.join(d, "copy_write"))
    fe, wr = counters(os.path.join(d, "fetch")), counters(os.path.join(d, "write"))
    copy_bytes = 1 << 30
    ck = "__amd_rocclr_copyBuffer"
    # counters are in KiB; scale so that the plain copy of copy_bytes reads / writes copy_bytes
    f_scale = copy_bytes / (cf[ck][1] * 1024) if ck in cf else None
    w_scale = copy_bytes / (cw[ck][1] * 1024) if ck in cw else None
    bench = None
    for line in open(os.path.join(d, "trace.log")) if os.path.exists(os.path.join(d, "trace.log")) else []:
        if line.startswith('{"metric"'):
            bench = json.loads(line)
    lines = ["| kernel | calls | avg us | total ms | % time |", "|---|---:|---:|---:|---:|"]
    tot = {}
    for n, r in enumerate(sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))):
        k = short_name(r["Name"])
        tot[k] = (int(r["Calls"]), float(r["AverageNs"]))
        if n >= 25:
            continue
        lines.append(f"| `{k}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.2f} |")
    traffic = {}
    tl = ["| kernel | launches (pmc) | FETCH B/launch | WRITE B/launch | HBM B/launch | algorithmic B/launch | "
          "HBM / algorithmic | HIP-event avg us | rocprof avg us |", "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    kt = (bench or {}).get("stencil_kernels", {})
    for k in sorted(set(fe) & set(wr)):
        if f_scale is None or w_scale is None:
            break
        fb = fe[k][1] * 1024 * f_scale
        wb = wr[k][1] * 1024 * w_scale
        alg = ev = None
        tk = timing_name(k)
        if tk in kt and kt[tk]["launches"]:
            alg = kt[tk]["GBs"] * kt[tk]["ms"] * 1e6 / kt[tk]["launches"]
            ev = kt[tk]["ms"] / kt[tk]["launches"] * 1e3
        traffic[tk] = dict(launches=fe[k][0], fetch_bytes=round(fb), write_bytes=round(wb),
                          hbm_bytes=round(fb + wb), algorithmic_bytes=round(alg) if alg else None)
        tl.append(f"| `{k}` | {fe[k][0]} | {fb:.4g} | {wb:.4g} | {fb + wb:.4g} | "
                  f"{alg:.4g} | {(fb + wb) / alg:.2f} | {ev:.1f} | {tot.get(k, (0, 0))[1] / 1e3:.1f} |"
                  if alg else f"| `{k}` | {fe[k][0]} | {fb:.4g} | {wb:.4g} | {fb + wb:.4g} | - | - | - | - |")
    src_hash = kernel_source_hash()
    with open(os.path.join(d, "stencil_traffic.json"), "w") as f:
        json.dump({"source_hash": src_hash, "fetch_scale": f_scale, "write_scale": w_scale, "kernels": traffic},
                  f, indent=1)
    with open(os.path.join(d, "summary.md"), "w") as f:
        f.write(HEADER)
        f.write(f"Stencil source hash: `{src_hash}`\n\n")
        if f_scale:
            f.write(f"Copy calibration (1 GiB device copy): FETCH_SIZE x {f_scale:.3f}, WRITE_SIZE x {w_scale:.3f} "
                    "give bytes.\n\n")
        if bench:
            f.write("Bench line of the traced run: value %.1f GB/s, roofline %s\n\n"
                    % (bench["value"], json.dumps(bench["roofline"])))
        f.write("Kernel trace (top 25 by total time, warm-up and timed steps together):\n\n")
        f.write("\n".join(lines) + "\n\nHBM traffic of the stencil kernels (counter passes):\n\n")
        f.write("\n".join(tl) + "\n")
        ut = units_table(d)
        if ut:
            f.write("\nVector-memory units of the stencil kernels (counter pass; fractions of "
                    f"{NCU} units x the dispatch's clocks, GRBM_GUI_ACTIVE / {NXCD}; reads and accesses summed over "
                    "the GPU):\n\n")
            f.write("\n".join(ut) + "\n")
    if not keep:
        for sub in ("trace", "fetch", "write", "copy_fetch", "copy_write", "units"):
            for p in glob.glob(os.path.join(d, sub, "**", "*"), recursive=True):
                if os.path.isfile(p):
                    os.remove(p)
    print(open(os.path.join(d, "summary.md")).read())


if __name__ == "__main__":
    main(sys.argv[1:])
