"""Profile summaries from rocprofv3 output.

summarize(db): per-kernel duration summary (count, total, mean, min, max in
microseconds) from a --kernel-trace SQLite database (rocpd format).

pmc_passes(csv): per-dispatch counter values from a --pmc run written with -f csv
(*_counter_collection.csv), cut into factorization passes (each pass starts at a
factor_init_kernel dispatch); prints every kernel's value and the sum of the factor
kernels of each complete pass.

copy_counter(csv, name): the counter summed over the dispatches of the copy kernel of a
calibration run.
"""
import csv
import glob
import sqlite3
import sys

FACTOR_KERNELS = ("factor_init_kernel", "factor_kernel", "factor_coop_kernel", "factor_spec_check_kernel",
                  "sepdense_kernel", "sepdense_prep_kernel", "sepdense_block_kernel", "sepdense_trail_kernel")


def summarize(path):
    con = sqlite3.connect(path)
    cur = con.cursor()
    tabs = [r[0] for r in cur.execute("select name from sqlite_master where type='table'")]
    kd = [t for t in tabs if t.startswith("rocpd_kernel_dispatch")][0]
    ks = [t for t in tabs if t.startswith("rocpd_info_kernel_symbol")][0]
    cols = [r[1] for r in cur.execute("pragma table_info(%s)" % ks)]
    namecol = "display_name" if "display_name" in cols else "kernel_name"
    q = ("select s.%s, count(*), sum(d.end - d.start), avg(d.end - d.start), min(d.end - d.start), "
         "max(d.end - d.start) from %s d join %s s on d.kernel_id = s.id group by s.%s "
         "order by sum(d.end - d.start) desc" % (namecol, kd, ks, namecol))
    rows = list(cur.execute(q))
    print("%-60s %6s %12s %12s %12s %12s" % ("kernel", "calls", "total_us", "mean_us", "min_us", "max_us"))
    for name, cnt, tot, avg, mn, mx in rows:
        print("%-60s %6d %12.1f %12.1f %12.1f %12.1f" % (name[:60], cnt, tot / 1e3, avg / 1e3, mn / 1e3, mx / 1e3))


def _rows(path):
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            yield (int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]))


def pmc_passes(path):
    per = {}
    for did, name, cname, val in _rows(path):
        key = (did, name)
        per[key] = per.get(key, 0.0) + val
        counter = cname
    disp = sorted(per.items())
    passes, cur = [], None
    for (did, name), val in disp:
        if "factor_init_kernel" in name:
            cur = []
            passes.append(cur)
        if cur is not None and any(k in name for k in FACTOR_KERNELS):
            cur.append((did, name, val))
    print("# %s  counter %s  (values as read, per dispatch)" % (path, counter))
    for i, ps in enumerate(passes):
        tot = sum(v for _, _, v in ps)
        print("pass %d: %d dispatches, sum %.1f" % (i, len(ps), tot))
        for did, name, val in ps:
            print("   %8d %-60s %14.1f" % (did, name[:60], val))
    return [sum(v for _, _, v in ps) for ps in passes]


def copy_counter(path, name_part):
    tot, n = 0.0, 0
    for did, name, cname, val in _rows(path):
        if name_part in name:
            tot += val
            n += 1
    return tot, n


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--pmc":
        pmc_passes(sys.argv[2])
        sys.exit(0)
    if len(sys.argv) > 3 and sys.argv[1] == "--copy":
        print(copy_counter(sys.argv[2], sys.argv[3]))
        sys.exit(0)
    for p in sys.argv[1:] or glob.glob("**/*_results.db", recursive=True):
        print("#", p)
        summarize(p)
