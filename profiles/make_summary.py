"""Write a short text summary of a rocprofv3 kernel-trace database.

    python profiles/make_summary.py <results.db> <title> <command> > profiles/<name>.txt
"""
import sqlite3
import sys


def main():
    db, title, cmd = sys.argv[1], sys.argv[2], sys.argv[3]
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels order by total_duration desc limit 20").fetchall()
    print(f"# {title}")
    print(f"# command: {cmd}")
    print("# times in microseconds (rocprofv3 --kernel-trace --stats, top_kernels view)")
    print(f"{'calls':>7} {'total_us':>12} {'avg_us':>10} {'pct':>6}  kernel")
    for name, calls, tot, avg, pct in rows:
        short = name.replace("trbdg::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        print(f"{calls:>7} {tot:>12.1f} {avg:>10.3f} {pct:>6.2f}  {short}")


if __name__ == "__main__":
    main()
