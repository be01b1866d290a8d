"""How much kernels on different hardware queues ran at the same time, from a rocprofv3
kernel trace (``--kernel-trace --output-format csv``: ``*_kernel_trace.csv``).

For every dispatch whose kernel name contains one of the given names, the time during
which at least one dispatch of another queue was running is summed, overall and per name
of the kernels it shared the chip with. Only dispatches that overlap some dispatch of
another queue are counted (the runs of one queue alone, e.g. the plain path, are left
out). Usage:

    python -m paper_2507_15703_amd.trace_overlap TRACE.csv k_pass_x k_pass_y k_pass_z k_gather
"""
import bisect
import csv
import sys
from collections import defaultdict


def short(name):
    base = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
    return base.split("::")[-1]


def load(path):
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), int(r["Queue_Id"]),
                         short(r["Kernel_Name"])))
    rows.sort()
    return rows


def overlap(rows, names):
    by_queue = defaultdict(list)
    for r in rows:
        by_queue[r[2]].append(r)
    # a queue runs its dispatches one after another: their ends are sorted with their starts
    ends = {q: [r[1] for r in lst] for q, lst in by_queue.items()}
    out = {}
    for name in names:
        total = shared = 0
        count = 0
        partners = defaultdict(int)
        for s, e, q, k in rows:
            if name not in k:
                continue
            # intervals of the other queues inside [s, e), merged
            iv = []
            for q2, lst in by_queue.items():
                if q2 == q:
                    continue
                i = bisect.bisect_right(ends[q2], s)
                while i < len(lst) and lst[i][0] < e:
                    s2, e2, _, k2 = lst[i]
                    iv.append((max(s, s2), min(e, e2), k2))
                    i += 1
            if not iv:
                continue
            count += 1
            total += e - s
            for a, b, k2 in iv:
                partners[k2] += b - a
            iv.sort()
            cs, ce = iv[0][0], iv[0][1]
            for a, b, _ in iv[1:]:
                if a > ce:
                    shared += ce - cs
                    cs, ce = a, b
                else:
                    ce = max(ce, b)
            shared += ce - cs
        out[name] = {"dispatches": count, "busy_us": total / 1e3, "shared_us": shared / 1e3,
                     "shared_frac": shared / total if total else 0.0,
                     "with": {k: round(v / 1e3, 1) for k, v in sorted(partners.items(), key=lambda t: -t[1])}}
    return out


def main():
    if len(sys.argv) < 3:
        print(__doc__)
        sys.exit(2)
    rows = load(sys.argv[1])
    for name, r in overlap(rows, sys.argv[2:]).items():
        print(f"{name}: {r['dispatches']} dispatches overlapping another queue, {r['busy_us']:.1f} us busy, "
              f"{r['shared_us']:.1f} us ({100 * r['shared_frac']:.1f} %) shared; with: {r['with']}")


if __name__ == "__main__":
    main()
