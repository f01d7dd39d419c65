"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite, written by
`rocprofv3 --kernel-trace --stats -d DIR -o run -- <command>`) into a short
per-kernel table: calls, total ms, average us, share of GPU kernel time.

Usage: python profiles/summarize.py DIR/run_results.db [N] > profiles/NAME.txt
"""
import re
import sqlite3
import sys


def short(name: str) -> str:
    name = name.replace("msc::(anonymous namespace)::", "").replace("void ", "")
    depth, out = 0, []
    for ch in name:  # drop the argument list, keep template arguments
        if ch == "(":
            depth += 1
        if depth == 0:
            out.append(ch)
        if ch == ")":
            depth -= 1
    return re.sub(r"\s+", " ", "".join(out)).strip()


def main():
    db = sys.argv[1]
    n = int(sys.argv[2]) if len(sys.argv) > 2 else 25
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    total = sum(r[2] for r in rows)
    print(f"{'kernel':44s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}")
    for r in rows[:n]:
        print(f"{short(r[0])[:44]:44s} {r[1]:7d} {r[2] / 1000:10.2f} {r[3]:10.1f} {r[4]:6.1f}")
    print(f"{'(all kernels)':44s} {sum(r[1] for r in rows):7d} {total / 1000:10.2f}")


if __name__ == "__main__":
    main()
