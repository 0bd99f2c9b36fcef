"""Short text summaries of rocprofv3 output (CSV), for the profile records
kept with the sources.

  python -m paper_1704_01144_amd.profile_summary stats DIR --command CMD
      per-kernel calls / total / average duration from DIR/*kernel_stats.csv

  python -m paper_1704_01144_amd.profile_summary counters --kernel SUBSTR \
      --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \
      --copy-bytes N --command CMD [--command CMD ...]
      mean FETCH_SIZE / WRITE_SIZE per dispatch of the kernels whose name
      contains SUBSTR, each scaled by what the same counter reads for a plain
      device-to-device copy of N bytes (the largest copy dispatch of the copy
      run), and the HBM bytes per launch that follow.  The record also holds
      the SHA-256 of the library sources, so that a reader can tell whether
      the kernels changed after the counters were taken.

  python -m paper_1704_01144_amd.profile_summary sq --kernel SUBSTR \
      --dir DIR [--dir DIR ...] --command CMD [--command CMD ...]
      per-wave means of SQ counters (each divided by SQ_WAVES of the same
      dispatches) for each kernel whose name contains a SUBSTR, from one
      or more --pmc runs that each also collected SQ_WAVES.

  python -m paper_1704_01144_amd.profile_summary gaps DIR --command CMD
      from DIR/*kernel_trace.csv: the dispatches split into bursts wherever
      the GPU idles for more than --split-ms (host synchronisation between
      the phases of a run); for the --top longest bursts, their span, the
      time with no kernel running, the idle gaps between kernels by length,
      and with --kernels K their K longest kernels.
"""
import argparse
import csv
import glob
import hashlib
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))


def source_digest():
    """SHA-256 over the native sources of the library (sorted by name)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(PKG, "csrc", "*"))):
        if os.path.isfile(p) and p.endswith((".hip", ".h", ".cpp")):
            h.update(os.path.basename(p).encode())
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _one(pattern):
    hits = glob.glob(pattern)
    if len(hits) != 1:
        raise SystemExit(f"expected one file for {pattern}, found {hits}")
    return hits[0]


def _short(name, width=90):
    name = name.replace("tafv::", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def stats_text(d, command, top=14):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "*kernel_stats.csv")))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"command: {command}", "",
           f"{'calls':>7} {'total ms':>10} {'avg us':>10} {'share':>6}  kernel"]
    for r in rows[:top]:
        out.append(f"{int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                   f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['Percentage']):5.1f}%  "
                   f"{_short(r['Kernel_Name'] if 'Kernel_Name' in r else r['Name'])}")
    out.append(f"{'':7} {total / 1e6:10.3f} {'':10} {'':6}  all kernels ({len(rows)} names)")
    return "\n".join(out) + "\n"


def _counter_rows(d, counter):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv")))))
    return [r for r in rows if r["Counter_Name"] == counter]


def _kernel_mean(d, counter, substr):
    vals = [float(r["Counter_Value"]) for r in _counter_rows(d, counter)
            if substr in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no {counter} dispatches of a kernel containing {substr!r} in {d}")
    names = {r["Kernel_Name"] for r in _counter_rows(d, counter) if substr in r["Kernel_Name"]}
    return sum(vals) / len(vals), len(vals), names


def _copy_kib(d, counter):
    rows = [r for r in _counter_rows(d, counter) if "copyBuffer" in r["Kernel_Name"]]
    if not rows:
        raise SystemExit(f"no copy dispatch in {d}")
    return max(float(r["Counter_Value"]) for r in rows)


def counters_text(a):
    f_kib, n_f, names = _kernel_mean(a.fetch, "FETCH_SIZE", a.kernel)
    w_kib, n_w, _ = _kernel_mean(a.write, "WRITE_SIZE", a.kernel)
    cf = _copy_kib(a.copy_fetch, "FETCH_SIZE")
    cw = _copy_kib(a.copy_write, "WRITE_SIZE")
    sf = a.copy_bytes / (cf * 1024.0)
    sw = a.copy_bytes / (cw * 1024.0)
    fetch_b = f_kib * 1024.0 * sf
    write_b = w_kib * 1024.0 * sw
    lines = [f"kernel: {a.kernel}"]
    lines += [f"kernel_name: {n}" for n in sorted(names)]
    lines += [f"command: {c}" for c in a.command]
    lines += [
        f"sources_sha256: {source_digest()}",
        f"dispatches_fetch: {n_f}",
        f"dispatches_write: {n_w}",
        f"fetch_kib_per_dispatch: {f_kib:.1f}",
        f"write_kib_per_dispatch: {w_kib:.1f}",
        f"copy_bytes: {a.copy_bytes}",
        f"copy_fetch_kib: {cf:.1f}",
        f"copy_write_kib: {cw:.1f}",
        f"fetch_scale: {sf:.4f}",
        f"write_scale: {sw:.4f}",
        f"traffic_fetch_bytes_per_launch: {fetch_b:.0f}",
        f"traffic_write_bytes_per_launch: {write_b:.0f}",
        f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}",
    ]
    return "\n".join(lines) + "\n"


def sq_text(a):
    """Per-wave SQ counter means of the named kernels over the given runs."""
    per = {}  # kernel -> counter -> [sum, dispatches]; waves per run
    for d in a.dir:
        rows = list(csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv")))))
        for sub in a.kernel:
            sel = [r for r in rows if sub in r["Kernel_Name"]]
            waves = sum(float(r["Counter_Value"]) for r in sel if r["Counter_Name"] == "SQ_WAVES")
            if not sel or waves == 0:
                raise SystemExit(f"no SQ_WAVES for a kernel containing {sub!r} in {d}")
            k = per.setdefault(sub, {})
            k.setdefault("SQ_WAVES", sum(1 for r in sel if r["Counter_Name"] == "SQ_WAVES"))
            for r in sel:
                if r["Counter_Name"] != "SQ_WAVES":
                    k[r["Counter_Name"]] = k.get(r["Counter_Name"], 0.0) + \
                        float(r["Counter_Value"]) / waves
    lines = [f"command: {c}" for c in a.command]
    lines.append(f"sources_sha256: {source_digest()}")
    lines.append("per-wave means (counter / SQ_WAVES over the same dispatches)")
    for sub in a.kernel:
        k = per[sub]
        lines.append(f"kernel: {sub} ({k['SQ_WAVES']} dispatches per run)")
        for name in sorted(x for x in k if x != "SQ_WAVES"):
            lines.append(f"  {name}: {k[name]:.1f}")
    return "\n".join(lines) + "\n"


def gaps_text(d, command, split_ms=1.0, top=2, kernels=0):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "*kernel_trace.csv")))))
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r.get("Kernel_Name", ""))
                for r in rows)
    bursts, cur, end = [], [], None
    for a, b, n in iv:
        if cur and a - end > split_ms * 1e6:
            bursts.append(cur)
            cur = []
        cur.append((a, b, n))
        end = b if end is None or not cur[:-1] else max(end, b)
    if cur:
        bursts.append(cur)
    edges = [2e3, 5e3, 10e3, 50e3, split_ms * 1e6]
    out = [f"command: {command}", f"bursts split at idle > {split_ms} ms: {len(bursts)}"]
    for k, bu in enumerate(sorted(bursts, key=lambda x: -(x[-1][1] - x[0][0]))[:top]):
        span = max(b for _, b, _ in bu) - bu[0][0]
        idle, last, counts = 0, bu[0][1], [0] * len(edges)
        for a, b, _ in bu[1:]:
            g = a - last
            if g > 0:
                idle += g
                counts[next(i for i, e in enumerate(edges) if g <= e)] += 1
            last = max(last, b)
        out.append(f"burst {k}: {len(bu)} dispatches, span {span / 1e6:.3f} ms, "
                   f"no kernel running {idle / 1e6:.3f} ms ({100.0 * idle / span:.1f}%)")
        lo = 0
        for e, n in zip(edges, counts):
            out.append(f"  idle gaps {lo / 1e3:g}-{e / 1e3:g} us: {n}")
            lo = e
        if kernels:
            per = {}
            for a, b, n in bu:
                t = per.setdefault(n, [0, 0])
                t[0] += 1
                t[1] += b - a
            out.append(f"  {'calls':>7} {'total ms':>10} {'avg us':>9}  kernel")
            for n, (c, t) in sorted(per.items(), key=lambda x: -x[1][1])[:kernels]:
                out.append(f"  {c:7d} {t / 1e6:10.3f} {t / c / 1e3:9.2f}  {_short(n, 80)}")
    return "\n".join(out) + "\n"


def read_record(path):
    """key: value lines of a counter record -> dict (repeated keys -> list)."""
    out = {}
    with open(path) as f:
        for line in f:
            if ":" not in line:
                continue
            k, v = line.split(":", 1)
            k, v = k.strip(), v.strip()
            if k in out:
                out[k] = out[k] if isinstance(out[k], list) else [out[k]]
                out[k].append(v)
            else:
                out[k] = v
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--command", required=True)
    s.add_argument("--top", type=int, default=14)
    c = sub.add_parser("counters")
    c.add_argument("--kernel", required=True)
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--copy-fetch", required=True)
    c.add_argument("--copy-write", required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--command", action="append", required=True)
    gp = sub.add_parser("gaps")
    gp.add_argument("dir")
    gp.add_argument("--command", required=True)
    gp.add_argument("--split-ms", type=float, default=1.0)
    gp.add_argument("--top", type=int, default=2)
    gp.add_argument("--kernels", type=int, default=0,
                    help="also list the longest kernels of each reported burst")
    q = sub.add_parser("sq")
    q.add_argument("--kernel", action="append", required=True)
    q.add_argument("--dir", action="append", required=True)
    q.add_argument("--command", action="append", required=True)
    a = ap.parse_args(argv)
    if a.what == "stats":
        sys.stdout.write(stats_text(a.dir, a.command, a.top))
    elif a.what == "sq":
        sys.stdout.write(sq_text(a))
    elif a.what == "gaps":
        sys.stdout.write(gaps_text(a.dir, a.command, a.split_ms, a.top, a.kernels))
    else:
        sys.stdout.write(counters_text(a))


if __name__ == "__main__":
    main()
