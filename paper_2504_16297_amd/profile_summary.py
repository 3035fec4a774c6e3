"""Turn rocprofv3 CSV output into the short text summaries kept with the
project, and read those summaries back.

    python -m paper_2504_16297_amd.profile_summary stats KERNEL_STATS_CSV --cmd "..." [--top 12] [--group RE]
    python -m paper_2504_16297_amd.profile_summary traffic --kernel ptsbe_pass_ \\
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv --copy-bytes B --cmd "..."
    python -m paper_2504_16297_amd.profile_summary counters COUNTER_CSV --kernel RE --cmd "..."

`traffic` averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) over the
dispatches of the named kernel and scales each by what the same counter reads
for a plain device copy of known size (the copy's bytes divided by its
counter), giving HBM bytes per dispatch.  The summary records the fingerprint
of the kernels the counters were taken with (`kernel_fingerprint`: the
generated source of every pass of the workload's plan, and the generic kernels'
source when a pass runs those), so a reader can tell when the kernels have
changed since.
"""

import argparse
import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_fingerprint(plan):
    """SHA-256 prefix over what runs on the device for the passes of `plan`:
    the generated source of every pass, and the generic tile kernels' source
    when some pass has no generated kernel (it then runs the generic ones)."""
    import ctypes as C
    from . import _lib as L
    h = hashlib.sha256()
    generic = False
    for p in range(plan.info["n_passes"]):
        n = C.c_size_t()
        L.check(L.lib().ptsbe_plan_pass_source(plan.handle, p, 0, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        L.check(L.lib().ptsbe_plan_pass_source(plan.handle, p, 0, buf, C.byref(n)))
        generic = generic or not buf.value
        h.update(buf.value)
    if generic:
        with open(os.path.join(HERE, "csrc", "kernels.hip"), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _short(name):
    m = re.search(r"(\w+)(<[^(]*>)?\(", name)
    base = m.group(1) if m else name[:60]
    if "float, 2u" in name:
        base += "<c64>"
    elif "double, 2u" in name:
        base += "<c128>"
    return base


def stats(path, top=12, group=None):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    if group:
        g = [r for r in rows if re.search(group, r["Name"])]
        calls = sum(int(r["Calls"]) for r in g)
        tot = sum(float(r["TotalDurationNs"]) for r in g)
        out.append("")
        out.append(f"group /{group}/: {len(g)} kernels, {calls} launches, {tot / 1e6:.3f} ms, "
                   f"average launch {tot / max(calls, 1) / 1e6:.4f} ms")
    return "\n".join(out)


def counter_per_dispatch(path, counter, kernel_regex):
    """Mean counter value (KiB) over the dispatches whose name matches."""
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter or not re.search(kernel_regex, r["Kernel_Name"]):
            continue
        d = r["Dispatch_Id"]
        vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"no {counter} rows for /{kernel_regex}/ in {path}")
    return sum(vals.values()) / len(vals), len(vals)


def traffic(a):
    copy_re = r"copyBuffer|copy_kernel|elementwise_kernel.*copy"
    cf, _ = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", copy_re)
    cw, _ = counter_per_dispatch(a.copy_write, "WRITE_SIZE", copy_re)
    fscale = a.copy_bytes / (cf * 1024.0)
    wscale = a.copy_bytes / (cw * 1024.0)
    f, nf = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel)
    w, nw = counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel)
    fb = f * 1024.0 * fscale
    wb = w * 1024.0 * wscale
    lines = [
        f"kernel: {a.kernel}",
        f"dispatches: fetch run {nf}, write run {nw}",
        f"FETCH_SIZE raw KiB/dispatch: {f:.1f}",
        f"WRITE_SIZE raw KiB/dispatch: {w:.1f}",
        f"copy calibration: {a.copy_bytes} bytes copied, FETCH_SIZE {cf:.1f} KiB -> scale {fscale:.4f}, "
        f"WRITE_SIZE {cw:.1f} KiB -> scale {wscale:.4f}",
        f"read_bytes_per_dispatch: {fb:.6g}",
        f"write_bytes_per_dispatch: {wb:.6g}",
        f"traffic_bytes_per_dispatch: {fb + wb:.6g}",
        f"kernel_fingerprint: {a.fingerprint}",
    ]
    return "\n".join(lines)


def counters(path, kernel_regex, note=""):
    """Totals of every counter over the dispatches whose name matches, and per
    wavefront when SQ_WAVES was collected."""
    tot, disp = {}, set()
    for r in csv.DictReader(open(path)):
        if not re.search(kernel_regex, r["Kernel_Name"]):
            continue
        disp.add(r["Dispatch_Id"])
        tot[r["Counter_Name"]] = tot.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    if not tot:
        raise SystemExit(f"no counter rows for /{kernel_regex}/ in {path}")
    waves = tot.get("SQ_WAVES")
    out = [f"kernels: /{kernel_regex}/{' (' + note + ')' if note else ''}, {len(disp)} dispatches"
           + (f", {waves:.4g} waves" if waves else ""), "",
           "| counter | total | per dispatch | per wave |", "|---|---|---|---|"]
    for c in sorted(tot):
        pw = f"{tot[c] / waves:.1f}" if waves else "-"
        out.append(f"| {c} | {tot[c]:.4g} | {tot[c] / len(disp):.4g} | {pw} |")
    return "\n".join(out)


def read_traffic(path):
    """(bytes per dispatch, kernel fingerprint) from a traffic summary, or None."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        m = re.match(r"\s*(traffic_bytes_per_dispatch|kernel_fingerprint):\s*(\S+)", line)
        if m:
            vals[m.group(1)] = m.group(2)
    if len(vals) != 2:
        return None
    return float(vals["traffic_bytes_per_dispatch"]), vals["kernel_fingerprint"]


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=12)
    s.add_argument("--group", default=None, help="regex: also report the combined average launch")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--fingerprint", required=True, help="kernel_fingerprint of the profiled plan "
                   "(python bench.py --fingerprint)")
    t.add_argument("--cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--kernel", required=True, help="regex of the kernel names to sum over")
    c.add_argument("--note", default="")
    c.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    if a.what == "stats":
        body = stats(a.csv, a.top, a.group)
    elif a.what == "traffic":
        body = traffic(a)
    else:
        body = counters(a.csv, a.kernel, a.note)
    sys.stdout.write(f"command: {a.cmd}\n\n{body}\n")


if __name__ == "__main__":
    main()
