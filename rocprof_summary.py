"""Summaries of rocprofv3 output databases (rocpd SQLite) as short text tables.

Kernel durations (from a `--kernel-trace --stats` run):

    python rocprof_summary.py trace <run_results.db> <command...>

Gaps between kernels of HIP-graph replays (from a `--kernel-trace` run of a program whose last
`replays` kernel issues are identical graph replays of one step; the kernels per replay are found
as the period of the trace's kernel-name sequence): the time the GPU runs no kernel between a
replay's first start and last end, as a fraction of that span, over all replays:

    python rocprof_summary.py gaps <run_results.db> <replays> <command...>

VALU issue per kernel from one PMC run (`--pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_WAVES SQ_BUSY_CYCLES`):
VALU instructions per wave, and the fraction of the VALU issue rate a kernel's launches use, i.e.
SQ_INSTS_VALU x 4 cycles (a wave64 instruction on a 16-lane SIMD) over 1024 SIMDs x the launch
time, both at the 2.4 GHz peak clock and at the clock the shader engines ran at (SQ_BUSY_CYCLES
per engine over the launch time, 32 engines); launches with fewer than `min_blocks` blocks are
left out:

    python rocprof_summary.py valu <run_results.db> <min_blocks> <command...>

HBM traffic per kernel from two PMC runs (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`) of a
program that first copies `copy_mib` MiB device-to-device: each counter is scaled by
(true bytes of that copy) / (what the counter reads for it). Also writes the traffic of one
step-kernel type to a JSON file keyed "<dir>:<type>:<workload>", with the SHA-256 of the kernel's
source (a comma-separated list: the kernel file and the headers it includes, hashed in that
order) so the figure is only used while that source is unchanged:

    python rocprof_summary.py pmc <fetch.db> <write.db> <copy_mib> \\
        <steps> <kernel substring> <key> <source file> <json out> <command...>
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
import re
import sqlite3
import sys


def short(name: str) -> str:
    name = re.sub(r"\(.*$", "", name.replace("(anonymous namespace)::", ""))
    return name.replace("grafx::", "").replace("void ", "")


def trace(db: str, cmd: str) -> None:
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                          "group by name order by sum(duration) desc"))
    total = sum(r[2] for r in rows)
    print(f"# rocprofv3 kernel summary\n# command: {cmd}\n# durations in microseconds\n")
    print(f"{'kernel':60s} {'calls':>6s} {'total_us':>10s} {'avg_us':>9s} {'share':>6s}")
    for name, n, tot, avg in rows:
        print(f"{short(name)[:60]:60s} {n:6d} {tot / 1e3:10.1f} {avg / 1e3:9.2f} "
              f"{100 * tot / total:5.1f}%")
    print(f"\n{'all kernels':60s} {sum(r[1] for r in rows):6d} {total / 1e3:10.1f}")


def gaps(db: str, replays: int, cmd: str) -> None:
    c = sqlite3.connect(db)
    rows = list(c.execute("select start, end, name from kernels order by start"))
    n = len(rows)
    names = [r[2] for r in rows]
    per = next(p for p in range(8, n // replays + 1)
               if all(names[n - (k + 1) * p:n - k * p] == names[n - p:]
                      for k in range(1, replays)))  # kernels per replay: the trace's period
    rows = rows[n - replays * per:]
    print(f"# rocprofv3 kernel trace: gaps between kernels inside HIP-graph replays\n"
          f"# command: {cmd}\n# {n} kernels traced; the last {replays} issues are graph "
          f"replays of {per} kernels each\n")
    print(f"{'replay':>6s} {'kernels':>8s} {'span_us':>10s} {'busy_us':>10s} {'gaps_us':>9s} "
          f"{'gap_frac':>8s} {'max_gap_us':>10s}")
    tot_span = tot_gap = 0.0
    for r in range(replays):
        seg = rows[r * per:(r + 1) * per]
        span = (max(e for _, e, _ in seg) - seg[0][0]) / 1e3
        busy, cur_s, cur_e, mx = 0.0, seg[0][0], seg[0][1], 0.0
        for s, e, _ in seg[1:]:
            if s > cur_e:
                busy += cur_e - cur_s
                mx = max(mx, (s - cur_e) / 1e3)
                cur_s, cur_e = s, e
            else:
                cur_e = max(cur_e, e)
        busy = (busy + cur_e - cur_s) / 1e3
        tot_span += span
        tot_gap += span - busy
        print(f"{r:6d} {len(seg):8d} {span:10.1f} {busy:10.1f} {span - busy:9.1f} "
              f"{(span - busy) / span:8.4f} {mx:10.2f}")
    print(f"\nall replays: gaps {tot_gap:.1f} us of {tot_span:.1f} us = {tot_gap / tot_span:.4f}")


def valu(db: str, min_blocks: int, cmd: str) -> None:
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, kernel_name, counter_name, value, duration, grid_size, "
                     "workgroup_size from counters_collection")
    disp: dict = collections.defaultdict(dict)
    for d, k, n, v, dur, gs, wg in rows:
        disp[d].update(k=k, dur=dur, blocks=gs // wg)
        disp[d][n] = v
    agg: dict = collections.defaultdict(lambda: collections.Counter())
    for x in disp.values():
        if x["blocks"] < min_blocks:
            continue
        a = agg[short(x["k"])]
        a["n"] += 1
        a["dur"] += x["dur"]
        for n in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_WAVES", "SQ_BUSY_CYCLES"):
            a[n] += x.get(n, 0)
    print(f"# rocprofv3 PMC summary: VALU issue per kernel (launches of at least {min_blocks} "
          f"blocks)\n# command: {cmd}\n")
    print(f"{'kernel':46s} {'calls':>5s} {'avg_us':>8s} {'valu/wave':>9s} {'lds/wave':>8s} "
          f"{'clk_GHz':>7s} {'issue@2.4':>9s} {'issue@clk':>9s}")
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["dur"]):
        if not a["SQ_WAVES"]:
            continue
        t = a["dur"] * 1e-9
        clk = a["SQ_BUSY_CYCLES"] / 32 / t / 1e9
        busy = a["SQ_INSTS_VALU"] * 4 / 1024 / t / 1e9  # GHz-equivalent of VALU issue
        print(f"{k[:46]:46s} {a['n']:5d} {a['dur'] / 1e3 / a['n']:8.1f} "
              f"{a['SQ_INSTS_VALU'] / a['SQ_WAVES']:9.0f} {a['SQ_INSTS_LDS'] / a['SQ_WAVES']:8.0f} "
              f"{clk:7.2f} {busy / 2.4:9.3f} {busy / clk:9.3f}")


def _counter(db: str, name: str):
    c = sqlite3.connect(db)
    return list(c.execute("select dispatch_id, kernel_name, value from counters_collection "
                          "where counter_name=? order by dispatch_id", (name,)))


def pmc(fetch_db: str, write_db: str, copy_mib: float, steps: int, kernel: str, key: str,
        source: str, json_out: str, cmd: str) -> None:
    f, w = _counter(fetch_db, "FETCH_SIZE"), _counter(write_db, "WRITE_SIZE")
    copy_f = max(v for _, n, v in f if "copyBuffer" in n)
    copy_w = max(v for _, n, v in w if "copyBuffer" in n)
    kib = copy_mib * 1024.0
    sf, sw = kib / copy_f, kib / copy_w
    agg = collections.defaultdict(lambda: [0, 0.0, 0.0])
    for (_, n, v), (_, n2, v2) in zip(f, w):
        if n != n2:
            raise SystemExit("the two PMC runs dispatched different kernels")
        a = agg[short(n)]
        a[0] += 1
        a[1] += v * sf
        a[2] += v2 * sw
    print(f"# rocprofv3 PMC summary: HBM traffic per kernel launch (scaled)\n# command: {cmd}")
    print(f"# calibration: a {copy_mib:g} MiB device copy reads FETCH_SIZE {copy_f:.1f} KiB and "
          f"WRITE_SIZE {copy_w:.1f} KiB -> scale fetch x{sf:.4f}, write x{sw:.4f}\n")
    print(f"{'kernel':50s} {'calls':>6s} {'fetch_KiB/call':>15s} {'write_KiB/call':>15s}")
    for k, (n, fe, wr) in sorted(agg.items(), key=lambda kv: -(kv[1][1] + kv[1][2])):
        print(f"{k[:50]:50s} {n:6d} {fe / n:15.1f} {wr / n:15.1f}")
    hits = [(k, v) for k, v in agg.items() if kernel in k]
    if len(hits) != 1:
        raise SystemExit(f"kernel substring {kernel!r} matches {len(hits)} kernels")
    name, (n, fe, wr) = hits[0]
    rec = json.load(open(json_out)) if os.path.exists(json_out) else {}
    rec[key] = {"kernel": name, "launches_per_step": n / steps,
                "fetch_bytes_per_launch": fe * 1024 / n, "write_bytes_per_launch": wr * 1024 / n,
                "bytes_per_launch": (fe + wr) * 1024 / n,
                "src_sha256": hashlib.sha256(b"".join(
                    open(f, "rb").read() for f in source.split(","))).hexdigest(),
                "command": cmd}
    with open(json_out, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    print(f"\n{name}: {(fe + wr) * 1024 / n / 1e6:.1f} MB per launch -> {json_out} [{key}]")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], " ".join(sys.argv[3:]))
    elif sys.argv[1] == "gaps":
        gaps(sys.argv[2], int(sys.argv[3]), " ".join(sys.argv[4:]))
    elif sys.argv[1] == "valu":
        valu(sys.argv[2], int(sys.argv[3]), " ".join(sys.argv[4:]))
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3], float(sys.argv[4]), int(sys.argv[5]), sys.argv[6],
            sys.argv[7], sys.argv[8], sys.argv[9], " ".join(sys.argv[10:]))
    else:
        raise SystemExit(__doc__)
