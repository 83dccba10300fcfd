"""Launch gaps of a stream of batched steps, from a rocprofv3 kernel trace.

    python -m paper_2602_23582_amd.trace_gaps <kernel_trace.csv> [summary.txt]

The trace (rocprofv3 --kernel-trace --output-format csv) is cut into ticks at
each k_sampler dispatch: one batched step per tick.  Per tick it measures the
span from the first kernel's start to the last kernel's end, the time the
GPU is busy (the union of the kernel intervals), the gaps between one kernel's
end and the next start inside the tick, and the pair kernel's share.  The
summary splits the ticks by span.
"""
import csv
import sys

import numpy as np


def ticks_of(path):
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    ticks, cur = [], []
    for s, e, n in rows:
        if "k_sampler" in n and cur:
            ticks.append(cur)
            cur = []
        cur.append((s, e, n))
    if cur:
        ticks.append(cur)
    return ticks


def summarise(ticks):
    spans, busy, gaps, nk, pair = [], [], [], [], []
    for t in ticks:
        st = min(s for s, _, _ in t)
        en = max(e for _, e, _ in t)
        iv = sorted((s, e) for s, e, _ in t)
        b = 0
        cs, ce = iv[0]
        for s, e in iv[1:]:
            if s > ce:
                b += ce - cs
                gaps.append(s - ce)
                cs, ce = s, e
            else:
                ce = max(ce, e)
        b += ce - cs
        spans.append(en - st)
        busy.append(b)
        nk.append(len(t))
        pair.append(sum(e - s for s, e, n in t if "k_pair" in n))
    spans, busy, pair = map(np.array, (spans, busy, pair))
    gaps = np.array(gaps) if gaps else np.zeros(1)
    lines = [
        f"ticks: {len(ticks)} (cut at each k_sampler dispatch), kernels per tick: median {int(np.median(nk))}",
        f"tick span (first kernel start to last kernel end), us: median {np.median(spans) / 1e3:.1f}, "
        f"p10 {np.percentile(spans, 10) / 1e3:.1f}, p90 {np.percentile(spans, 90) / 1e3:.1f}",
        f"GPU busy within a tick (union of kernel intervals) / span: {busy.sum() / spans.sum():.3f} overall, "
        f"median per tick {np.median(busy / spans):.3f}",
        f"gaps between consecutive kernels inside a tick, us: median {np.median(gaps) / 1e3:.1f}, "
        f"p90 {np.percentile(gaps, 90) / 1e3:.1f}, total {gaps.sum() / 1e6:.1f} ms",
        f"pair-kernel time / span: {pair.sum() / spans.sum():.3f}",
    ]
    for lo, hi in ((0, 0.3e6), (0.3e6, 2e6), (2e6, 1e12)):
        m = (spans >= lo) & (spans < hi)
        if m.any():
            lines.append(f"ticks with span in [{lo / 1e3:.0f}, {hi / 1e3:.0f}) us: {int(m.sum())}, "
                         f"busy/span {busy[m].sum() / spans[m].sum():.3f}, median span {np.median(spans[m]) / 1e3:.1f} us")
    return "\n".join(lines) + "\n"


def main(argv):
    if len(argv) < 2:
        raise SystemExit(__doc__)
    text = summarise(ticks_of(argv[1]))
    if len(argv) > 2:
        with open(argv[2], "w") as fh:
            fh.write(text)
    sys.stdout.write(text)


if __name__ == "__main__":
    main(sys.argv)
