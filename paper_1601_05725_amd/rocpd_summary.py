"""Per-kernel duration summary (count, total, mean, min, max in microseconds) from a
rocprofv3 --kernel-trace SQLite database (rocpd format)."""
import glob
import sqlite3
import sys


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


if __name__ == "__main__":
    for p in sys.argv[1:] or glob.glob("gpurun_out/**/*_results.db", recursive=True):
        print("#", p)
        summarize(p)
