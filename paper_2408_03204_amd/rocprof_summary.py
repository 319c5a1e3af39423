"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) into a short text table:
per kernel, calls, total and average duration (us), share of GPU time.

    python -m paper_2408_03204_amd.rocprof_summary <run_results.db> <command> > profiles/<name>.txt
"""
import re
import sqlite3
import sys


def short(name: str) -> str:
    name = re.sub(r"\(.*$", "", name.replace("(anonymous namespace)::", ""))
    return name.replace("grafx::", "").replace("void ", "")


def main(db: str, cmd: str) -> None:
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


if __name__ == "__main__":
    main(sys.argv[1], " ".join(sys.argv[2:]))
