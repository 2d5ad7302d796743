"""Write a short text summary of a rocprofv3 kernel-statistics file.

    python profiles/make_summary.py <kernel_stats.csv> <title> <command>

Reads the CSV that `rocprofv3 --kernel-trace --stats --output-format csv`
writes (`*_kernel_stats.csv`) and prints the 20 most expensive kernels.
"""
import csv
import sys


def main():
    path, title, cmd = sys.argv[1], sys.argv[2], sys.argv[3]
    rows = list(csv.DictReader(open(path)))
    print(f"# {title}")
    print(f"# command: {cmd}")
    print("# rocprofv3 --kernel-trace --stats (kernel_stats.csv); times in microseconds")
    print(f"{'calls':>7} {'total_us':>12} {'avg_us':>10} {'pct':>6}  kernel")
    for r in rows[:20]:
        name = r["Name"].replace("trbdg::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        print(f"{int(r['Calls']):>7} {float(r['TotalDurationNs']) / 1e3:>12.1f} "
              f"{float(r['AverageNs']) / 1e3:>10.3f} {float(r['Percentage']):>6.2f}  {name}")


if __name__ == "__main__":
    main()
