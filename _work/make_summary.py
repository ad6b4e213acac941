"""Write short text summaries of rocprofv3 output for profiles/.

  python profiles/make_summary.py trace <results.db> "<command>" [name filter]
      kernel-trace statistics (top kernels and per-dispatch durations),
      optionally only kernels whose name contains the filter (alternatives
      separated by "|")
  python profiles/make_summary.py traffic <fetch.csv> <write.csv> <kernel-sha> "<commands>"
      HBM bytes per solve launch from FETCH_SIZE / WRITE_SIZE passes, each
      scaled by what the same counter reads for a 1 GiB device copy
"""
import csv
import sqlite3
import sys

GIB_KIB = 1 << 20  # FETCH_SIZE / WRITE_SIZE count KiB


def trace(db, cmd, only=""):
    c = sqlite3.connect(db)
    alts = [a for a in only.split("|") if a]

    def keep(name):
        return not alts or any(a in name for a in alts)

    print(f"command: `{cmd}`\n")
    if only:
        print(f"kernels whose name contains `{only}`\n")
    print("| kernel | calls | total ms | average ms | % |")
    print("|---|---|---|---|---|")
    # top_kernels reports microseconds, the kernels table nanoseconds.
    for name, calls, tot, avg, pct in c.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"):
        if not keep(name):
            continue
        print(f"| {name[:90]} | {calls} | {tot / 1e3:.3f} | {avg / 1e3:.4f} | {pct:.2f} |")
    rows = list(c.execute("select name, duration, grid_x, workgroup_x, vgpr_count, "
                          "accum_vgpr_count, scratch_size from kernels order by start"))
    solve = [r for r in rows if any(k in r[0] for k in ("solve_kernel", "vjp_kernel",
                                                        "stiff_kernel", "sens_kernel"))
             and keep(r[0])]
    if solve:
        print("\nper dispatch (solver kernels, at most 12): duration ms, grid, block, vgpr, agpr, "
              "scratch")
        for r in solve[:12]:
            print(f"- {r[0][:70]}: {r[1] / 1e6:.3f} ms, grid {r[2]}, block {r[3]}, "
                  f"vgpr {r[4]}, agpr {r[5]}, scratch {r[6]}")


def _counter(path, name):
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == name:
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    agg = {}
    for d, k, v in out:
        agg.setdefault(d, [k, 0.0])[1] += v
    return [(d, k, v) for d, (k, v) in sorted(agg.items())]


def traffic(fetch_csv, write_csv, sha, cmds):
    f = _counter(fetch_csv, "FETCH_SIZE")
    w = _counter(write_csv, "WRITE_SIZE")

    def pick(rows, key):
        return [r for r in rows if key(r[1])]

    copy_f = pick(f, lambda k: "copy" in k.lower() or "elementwise" in k.lower())
    copy_w = pick(w, lambda k: "copy" in k.lower() or "elementwise" in k.lower())
    solve_f = pick(f, lambda k: "solve_kernel" in k)
    solve_w = pick(w, lambda k: "solve_kernel" in k)
    # the copy reads and writes 1 GiB: the largest copy-like dispatch is it
    cf = max(v for _, _, v in copy_f)
    cw = max(v for _, _, v in copy_w)
    kf, kw = GIB_KIB / cf, GIB_KIB / cw
    sf, sw = solve_f[-1][2], solve_w[-1][2]
    total = (sf * kf + sw * kw) * 1024
    print(f"commands: {cmds}\n")
    print(f"kernel source sha: {sha}")
    print(f"copy of 1 GiB: FETCH_SIZE {cf:.0f} KiB (scale {kf:.4f}), "
          f"WRITE_SIZE {cw:.0f} KiB (scale {kw:.4f})")
    print(f"solve kernel: FETCH_SIZE {sf:.0f} KiB, WRITE_SIZE {sw:.0f} KiB")
    print(f"HBM bytes per launch: {total:.6e}")
    print(f"(read {sf * kf * 1024:.4e} B, written {sw * kw * 1024:.4e} B)")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else "")
    else:
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
