"""Plain-text summaries of rocprofv3 result databases (rocpd SQLite) for this
library's kernels.

    python -m paper_1912_05371_amd.profile_summary trace DB [--match wacm]
        per-kernel dispatch count and duration statistics of a kernel trace
    python -m paper_1912_05371_amd.profile_summary counters DB [DB ...] [--match wacm]
        [--copy-gib G]
        per-kernel mean of every collected counter; with --copy-gib, the
        FETCH_SIZE / WRITE_SIZE scale factors implied by bench.py's copy probe
        (a torch.neg kernel that reads and writes G GiB once each)
    python -m paper_1912_05371_amd.profile_summary dispatches DB [--match stage_kernel]
        one line per matching dispatch: kernel and counter values, in order
    python -m paper_1912_05371_amd.profile_summary traffic DBFETCH DBWRITE --copy-gib G
        --dtype D --schedule KEY --last N
        HBM bytes per stage-kernel launch, the mean over the last N stage
        launches (the timed steps) of a `bench.py --no-graph --dtype D
        --schedule KEY` run under rocprofv3 --pmc (FETCH_SIZE in one run,
        WRITE_SIZE in another), each counter scaled by the copy probe, as the
        machine-readable block bench.py reads back.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
STAGE_SOURCES = ("csrc/kernels.hip", "csrc/resolve.h", "csrc/wacm_internal.h")


def stage_source_sha1() -> str:
    """Hash of the sources the stage kernel is compiled from: counters taken
    with other sources no longer describe the kernel."""
    h = hashlib.sha1()
    for rel in STAGE_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    n = re.sub(r"\(.*$", "", name)
    return n.replace("void ", "").strip()


def kernel_rows(db: str, match: str):
    c = sqlite3.connect(db)
    rows = c.execute("select name, start, end from kernels order by start").fetchall()
    return [(short_name(n), (e - s) * 1e-3) for n, s, e in rows if match in n]


def is_copy_probe(name: str) -> bool:
    """bench.py's copy probe is torch.neg on doubles."""
    return "neg_kernel" in name


def dispatch_counters(db: str, match: str):
    """[(kernel short name, {counter: value})] in dispatch order."""
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, name, counter_name, counter_value from pmc_events "
                     "order by dispatch_id").fetchall()
    out, last = [], None
    for did, name, cn, v in rows:
        if match not in name and not is_copy_probe(name):
            continue
        if did != last:
            out.append((short_name(name), {}))
            last = did
        d = out[-1][1]
        d[cn] = d.get(cn, 0.0) + float(v)
    return out


def trace_table(db: str, match: str) -> str:
    agg = {}
    for n, us in kernel_rows(db, match):
        a = agg.setdefault(n, [0, 0.0, 1e30, 0.0])
        a[0] += 1
        a[1] += us
        a[2] = min(a[2], us)
        a[3] = max(a[3], us)
    lines = [f"{'kernel':72s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} "
             f"{'total_ms':>9s}"]
    for n, (k, t, mn, mx) in sorted(agg.items(), key=lambda x: -x[1][1]):
        lines.append(f"{n[:72]:72s} {k:6d} {t / k:10.1f} {mn:10.1f} {mx:10.1f} {t / 1e3:9.2f}")
    return "\n".join(lines)


def copy_factors(disp, copy_gib: float):
    """Scale factors that make the copy probe's counters read its true bytes."""
    neg = [d for n, d in disp if is_copy_probe(n)]
    if not neg:
        return {}
    true_kib = copy_gib * (1 << 20)
    f = {}
    for cn in ("FETCH_SIZE", "WRITE_SIZE"):
        vals = [d[cn] for d in neg if cn in d]
        if vals:
            f[cn] = true_kib / (sum(vals) / len(vals))
    return f


def counter_table(dbs, match: str, copy_gib: float) -> str:
    lines = []
    for db in dbs:
        disp = dispatch_counters(db, match)
        fac = copy_factors(disp, copy_gib) if copy_gib else {}
        agg = {}
        for n, d in disp:
            for cn, v in d.items():
                a = agg.setdefault((n, cn), [0, 0.0])
                a[0] += 1
                a[1] += v
        lines.append(f"{os.path.basename(os.path.dirname(db)) or db}:")
        for (n, cn), (k, s) in sorted(agg.items()):
            extra = ""
            if cn in fac:
                extra = f"  x{fac[cn]:.3f} = {s / k * fac[cn] * 1024 / 1e9:.3f} GB"
            lines.append(f"  {n[:64]:64s} {cn:22s} n={k:5d} mean={s / k:16.1f}{extra}")
        if fac:
            lines.append("  copy-probe scale factors: " +
                         ", ".join(f"{k} x{v:.4f}" for k, v in fac.items()))
    return "\n".join(lines)


def stage_traffic(db_fetch: str, db_write: str, copy_gib: float, last: int):
    """Mean scaled FETCH_SIZE and WRITE_SIZE bytes over the last `last`
    stage-kernel launches, and the scale factors."""
    out, fac = {}, {}
    for cn, db in (("FETCH_SIZE", db_fetch), ("WRITE_SIZE", db_write)):
        disp = dispatch_counters(db, "stage_kernel")
        f = copy_factors(disp, copy_gib)
        if cn not in f:
            raise SystemExit(f"{db}: no copy-probe dispatch with {cn}")
        fac[cn] = f[cn]
        st = [d[cn] for n, d in disp if "stage_kernel" in n]
        if len(st) < last:
            raise SystemExit(f"{db}: {len(st)} stage launches, fewer than {last}")
        out[cn] = sum(st[-last:]) / last * fac[cn] * 1024
    return out, fac


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("mode", choices=["trace", "counters", "dispatches", "traffic"])
    ap.add_argument("dbs", nargs="+")
    ap.add_argument("--match", default="wacm")
    ap.add_argument("--copy-gib", type=float, default=0.0)
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--schedule", default="")
    ap.add_argument("--last", type=int, default=0)
    a = ap.parse_args(argv)
    if a.mode == "trace":
        for db in a.dbs:
            print(trace_table(db, a.match))
    elif a.mode == "counters":
        print(counter_table(a.dbs, a.match, a.copy_gib))
    elif a.mode == "dispatches":
        for db in a.dbs:
            for i, (n, d) in enumerate(dispatch_counters(db, a.match)):
                print(f"{i:5d} {n[:60]:60s} " +
                      " ".join(f"{k}={v:.0f}" for k, v in sorted(d.items())))
    else:
        if len(a.dbs) != 2 or not a.copy_gib or not a.schedule or a.last <= 0:
            raise SystemExit("traffic needs DBFETCH DBWRITE, --copy-gib, --schedule, --last")
        v, fac = stage_traffic(a.dbs[0], a.dbs[1], a.copy_gib, a.last)
        key = ",".join(sorted(a.schedule.split(",")))
        print(f"copy-probe scale factors: FETCH_SIZE x{fac['FETCH_SIZE']:.4f}, "
              f"WRITE_SIZE x{fac['WRITE_SIZE']:.4f}")
        print("traffic-data")
        print(f"source_sha1 {stage_source_sha1()}")
        print(f"{a.dtype} {key} fetch {v['FETCH_SIZE']:.0f} write {v['WRITE_SIZE']:.0f}")
        print("end-traffic-data")
    return 0


if __name__ == "__main__":
    sys.exit(main())
