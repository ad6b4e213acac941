"""Write a short text summary of a rocprofv3 kernel-trace database.

Usage: python profiles/make_summary.py <results.db> "<command that made it>" > summary.md
"""
import sqlite3
import sys


def main(db, cmd):
    c = sqlite3.connect(db)
    print(f"command: `{cmd}`\n")
    print("| kernel | calls | total ms | average ms | % |")
    print("|---|---|---|---|---|")
    # top_kernels reports microseconds, the kernels table nanoseconds.
    for name, calls, tot, avg, pct in c.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"):
        print(f"| {name[:90]} | {calls} | {tot / 1e3:.3f} | {avg / 1e3:.4f} | {pct:.2f} |")
    rows = list(c.execute("select name, duration, grid_x, workgroup_x, vgpr_count, "
                          "accum_vgpr_count, scratch_size from kernels order by start"))
    solve = [r for r in rows if "solve_kernel" in r[0] or "vjp_kernel" in r[0]]
    if solve:
        print("\nper dispatch (solve/vjp kernels): duration ms, grid, block, vgpr, agpr, scratch")
        for r in solve:
            print(f"- {r[0][:60]}: {r[1] / 1e6:.3f} ms, grid {r[2]}, block {r[3]}, "
                  f"vgpr {r[4]}, agpr {r[5]}, scratch {r[6]}")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
