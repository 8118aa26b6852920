"""Summarise a rocprofv3 kernel trace (the ``*_results.db`` SQLite file that
``rocprofv3 --kernel-trace`` writes) as a Markdown table.

Usage: python -m paper_2307_01117_amd.trace_summary DB [--kernel TEXT]
           [--skip N] [--take M] [--pmc]

Per kernel: dispatches, average / median / min / max duration and share of
the GPU time.  With ``--kernel`` the dispatches of the first kernel whose name
contains TEXT are also averaged over the index range [skip, skip + take) in
launch order -- for a benchmark that launches it W times in its warm-up and K
times in its timed region, ``--skip W --take K`` averages the timed launches
alone.  Gaps: idle time between the end of one dispatch and the start of the
next.  With ``--pmc`` the counters a ``--pmc`` run recorded are averaged per
kernel instead.
"""
from __future__ import annotations

import argparse
import sqlite3
import statistics


def kernel_rows(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    con.close()
    return rows


def pmc_rows(db):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, value from counters_collection"
                       ).fetchall()
    con.close()
    return rows


def short(name, n=100):
    return name if len(name) <= n else name[:n] + "..."


def summarise(db, kernel=None, skip=0, take=None):
    rows = kernel_rows(db)
    per = {}
    for name, s, e in rows:
        per.setdefault(name, []).append(e - s)
    total = sum(sum(v) for v in per.values()) or 1
    out = ["| kernel | calls | avg (us) | median (us) | min (us) | max (us) | share of GPU time |",
           "|---|---|---|---|---|---|---|"]
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| `{short(name)}` | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | "
                   f"{statistics.median(v) / 1e3:.2f} | {min(v) / 1e3:.2f} | "
                   f"{max(v) / 1e3:.2f} | {100 * sum(v) / total:.2f} % |")
    if kernel:
        names = [n for n in per if kernel in n]
        if names:
            v = per[names[0]]
            sel = v[skip:skip + take if take else None]
            if sel:
                out.append("")
                out.append(f"`{short(names[0])}`, dispatches {skip} to {skip + len(sel) - 1} "
                           f"(launch order) of {len(v)}: avg {sum(sel) / len(sel) / 1e3:.2f} us, "
                           f"median {statistics.median(sel) / 1e3:.2f} us, "
                           f"min {min(sel) / 1e3:.2f} us, max {max(sel) / 1e3:.2f} us")
    gaps = [rows[i + 1][1] - rows[i][2] for i in range(len(rows) - 1)]
    gaps = [g for g in gaps if g > 0]
    if gaps:
        gaps.sort()
        out.append("")
        out.append(f"Idle gaps between consecutive dispatches: {len(gaps)} of {len(rows) - 1} "
                   f"positive; median {statistics.median(gaps) / 1e3:.2f} us, "
                   f"90th percentile {gaps[int(0.9 * (len(gaps) - 1))] / 1e3:.2f} us")
    return "\n".join(out)


def summarise_pmc(db):
    per = {}
    for name, counter, value in pmc_rows(db):
        per.setdefault((name, counter), []).append(value)
    out = ["| kernel | counter | dispatches | average per dispatch |", "|---|---|---|---|"]
    for (name, counter), v in sorted(per.items()):
        out.append(f"| `{short(name)}` | {counter} | {len(v)} | {sum(v) / len(v):.6g} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--skip", type=int, default=0)
    ap.add_argument("--take", type=int, default=0)
    ap.add_argument("--pmc", action="store_true")
    a = ap.parse_args()
    if a.pmc:
        print(summarise_pmc(a.db))
    else:
        print(summarise(a.db, a.kernel, a.skip, a.take or None))


if __name__ == "__main__":
    main()
