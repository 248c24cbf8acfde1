"""Summarise a rocprofv3 kernel trace (rocpd SQLite database) as a markdown table.

Usage: python profiles/make_summary.py <results.db> <title> <command> [limit]
"""
import re
import sqlite3
import sys


def main():
    db, title, command = sys.argv[1], sys.argv[2], sys.argv[3]
    limit = int(sys.argv[4]) if len(sys.argv) > 4 else 30
    cur = sqlite3.connect(db).cursor()
    out = [f"# {title}", "", "Command (repository root, GPU box):", f"    {command}", "",
           "Durations in microseconds, from the rocpd `top_kernels` view of the run's database.", "",
           "| kernel | calls | total us | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, total, avg, pct in cur.execute(f"select * from top_kernels limit {limit}"):
        name = name.replace("spai::(anonymous namespace)::", "").replace("void ", "")
        name = name.replace("spai::", "")
        name = re.sub(r"\(.*$", "", name)
        out.append(f"| {name} | {calls} | {total:.0f} | {avg:.1f} | {pct:.1f} |")
    print("\n".join(out))


if __name__ == "__main__":
    main()
