"""Benchmark of the packet-transport hot path on one MI355X.

    python bench.py [--gpus 1] [--steps 10] [--warmup 1]
    python bench.py --workload batched [--steps 3]
    python bench.py --workload served [--duration 10]
    python bench.py --workload copy      (plain 1 GiB device copies: the
                                          reference for HBM byte counters)
    python bench.py --workload virtual [--n-virtual 3]
                                         (the final spectrum iteration with
                                          virtual packets, section 2.9)
    python bench.py --workload macroatom (macroatom vs downbranch line modes
                                          on the 30-shell 2e4-line atom)
    python bench.py --workload plasma [--nlte]
                                         (iterations with the plasma update of
                                          sections 2.3 and 2.5 between them;
                                          --nlte: Mg II, Si II, S II, Ca II
                                          analogues in NLTE excitation)

One step is one Monte Carlo iteration of the paper-scale scatter model
(20 shells 10000-25000 km/s at 13 d, 3e5 lines, 1e6 packets; Kerzendorf & Sim
2014 sections 2.4-2.8): reset, injection + propagation of every packet,
estimator normalisation and the T_R / W / T_inner update, all on the device,
with T_inner carried from one iteration to the next on the device.  The K
timed steps are iterations 0..K-1 starting from T_inner = 9000 K.

Prints ONE JSON line.  The value is packet interactions (line events plus
Thomson scatterings) per second over the timed iterations.  The roofline
entry prices the transport pass (the lane-per-packet kernel, the hand-off
ordering and the group kernel of the handed-off histories, timed together by
the library's HIP events on the launch stream) at its algorithmic bytes --
16 B per line passed (nu_k and tau_S read), 24 B per flight segment (shell
radii and density), 96 B per packet (its state written and read once) --
against the HBM peak; `traffic` is the measured HBM bytes per transport pass
from the committed hardware-counter summary when it was taken on the current
kernel source (else null).  Its `atomic` entry sets the pass's atomic
requests at the L2 (J_blue, J, nu-bar and spectrum tallies; TCC_ATOMIC from
the committed counter summary) per second against the request rate the
device sustains in the two tally patterns: their FP64 add rates, measured in
the same run, times the requests per add the calibration counters read.  Its
`valu` entry sets the pass's wave64 VALU instructions (SQ_INSTS_VALU from the
same summary) per second against the issue peak, one per 4 cycles per SIMD:
the resource the pass is bound by.  The `batched` entry is the 64-model mix
in one autotuned multi-model launch against 64 single-model launches
(models/s; also with the library's default tuning).
The CPU baseline times the FP64 oracle on a bounded packet sample of the
same iterations: an equal share of --cpu-sample packets from every timed
iteration, each at the iteration number and T_inner the device used, once
on one host core and once split over --cpu-procs oracle processes on
disjoint packet-id ranges (the host's CPU share); it reports the latter,
with the single-core figure inside.

    python bench.py --workload atomics   (the device's FP64 atomic-add rates)
    python bench.py --workload critical  (the longest history of the last of
                                          --steps iterations, run alone)
    python bench.py --profile-summary DB [DB ...]
                                         (per-kernel counter summary of
                                          rocprofv3 --pmc databases)
    python bench.py --traffic-summary OUT BENCH_FETCH_DB BENCH_WRITE_DB \
                    COPY_FETCH_DB COPY_WRITE_DB BENCH_LINE [--commands ...]
    python bench.py --counter-summary OUT BENCH_LINE ATOMICS_DB BENCH_DB... \
                    [--commands ...]     (the committed summaries the
                                          roofline's traffic and atomic
                                          entries read)
    python bench.py --trace-summary DB [BENCH_LINE]
                                         (kernel-trace summary per pass)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes of the transport pass
BYTES_PER_LINE_PASS = 16.0   # nu_k and tau_S of every line passed
BYTES_PER_SEGMENT = 24.0     # shell radii and electron density
BYTES_PER_PACKET = 96.0      # packet state written once and read once
KERNEL_SOURCE = os.path.join(ROOT, "paper_1401_5469_amd", "csrc", "smc_kernels.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_scatter-20shell-300kline.json")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "counters_scatter-20shell-300kline.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample", type=int, default=400_000,
                    help="packets the oracle runs for the CPU baseline, shared equally "
                         "among the timed iterations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="oracle processes of the all-cores CPU baseline (the host's CPU share)")
    ap.add_argument("--cpu-worker", metavar="JOBS", help=argparse.SUPPRESS)
    ap.add_argument("--no-critical-path", action="store_true",
                    help="skip the untimed replay of the longest history (profiling runs)")
    ap.add_argument("--no-jblue", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-plain entry of the paper-scale line (profiling runs)")
    ap.add_argument("--profile-summary", nargs="+", metavar="DB",
                    help="print per-kernel summaries of rocprofv3 --pmc result databases")
    ap.add_argument("--traffic-summary", nargs=6, metavar="PATH",
                    help="write the HBM traffic summary: OUT BENCH_FETCH_DB BENCH_WRITE_DB "
                         "COPY_FETCH_DB COPY_WRITE_DB BENCH_LINE")
    ap.add_argument("--counter-summary", nargs="+", metavar="PATH",
                    help="write the counter summary: OUT BENCH_LINE ATOMICS_DB BENCH_DB...")
    ap.add_argument("--trace-summary", nargs="+", metavar="PATH",
                    help="print the kernel-trace summary: DB [BENCH_LINE]")
    ap.add_argument("--profile-last", type=int, default=0,
                    help="with --profile-summary: also list the last N dispatches one by one")
    ap.add_argument("--profile-kernel", default="",
                    help="with --profile-last: only dispatches whose kernel name contains this")
    ap.add_argument("--commands", nargs="*", help="commands recorded in a summary")
    ap.add_argument("--atomic-rounds", type=int, default=256,
                    help="rounds per lane of the atomics workload (counter summary)")
    ap.add_argument("--workload", default="paper-scale",
                    choices=["paper-scale", "batched", "served", "copy", "virtual",
                             "macroatom", "plasma", "atomics", "critical"])
    ap.add_argument("--n-virtual", type=int, default=3,
                    help="virtual packets per packet launch in the virtual mode")
    ap.add_argument("--nlte", action="store_true",
                    help="plasma mode: NLTE excitation for four ions, J_b from J_blue")
    ap.add_argument("--models", type=int, default=64, help="models in the batched mix")
    ap.add_argument("--duration", type=float, default=60.0,
                    help="seconds of Poisson arrivals (20 per second) in the served mode")
    ap.add_argument("--served-modes", default="stream,step,plain",
                    help="served mode: comma-separated paths among stream, step, plain")
    ap.add_argument("--streams", type=int, default=4,
                    help="launch streams of the stream server")
    ap.add_argument("--max-active", type=int, default=128,
                    help="requests a server keeps admitted at once (the rest queue in "
                         "arrival order)")
    ap.add_argument("--max-cohort", type=int, default=1024,
                    help="requests one launch of the stream server takes at most")
    ap.add_argument("--plain-requests", type=int, default=200,
                    help="requests (in arrival order) the plain path serves")
    ap.add_argument("--budget-gb", type=float, default=200.0,
                    help="device-memory admission budget of the served mode")
    return ap.parse_args()


def _current_summary(path):
    """A committed hardware-counter summary, if it was taken on the kernel
    source that is built now (else None)."""
    import hashlib

    try:
        with open(path) as f:
            summ = json.load(f)
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    return summ if summ.get("kernel_source_sha256") == sha else None


def measured_traffic():
    """HBM bytes per transport pass from the hardware-counter summary."""
    summ = _current_summary(TRAFFIC_SUMMARY)
    return summ.get("bytes_per_transport_pass") if summ else None


def measured_atomics():
    """The pass's L2 atomic requests from the counter summary (per pass) and
    the requests per FP64 atomic add of each calibration pattern."""
    summ = _current_summary(COUNTER_SUMMARY)
    if not summ:
        return None
    return {"requests_per_pass": summ["per_pass"]["TCC_ATOMIC_sum"],
            "requests_per_add": {k: v["TCC_ATOMIC_sum_per_add"]
                                 for k, v in summ["atomic_calibration"].items()}}


def measured_valu():
    """The pass's wave64 VALU instructions from the counter summary (per
    pass, and the part of them in the kernel of the handed-off histories)."""
    summ = _current_summary(COUNTER_SUMMARY)
    if not summ:
        return None
    solo = summ["per_kernel"].get("solo_kernel", {}).get("SQ_INSTS_VALU")
    return {"per_pass": summ["per_pass"]["SQ_INSTS_VALU"], "handed_off_kernel": solo,
            "segments_per_pass": summ["segments_per_pass"]}


def valu_entry(pass_ms):
    """The pass's VALU issue rate against the device's: the resource the
    handed-off histories' kernel saturates while thousands of long histories
    run (its FP64 chains are uniform per history, so every segment costs the
    same wave64 instructions whatever the lanes do)."""
    v = measured_valu()
    peak = valu_peak()
    if not v:
        return {"achieved": None, "peak": peak, "unit": "wave64 VALU instructions/s",
                "frac": None, "source": "committed counter summary (null: kernel source changed)"}
    rate = v["per_pass"] / (pass_ms * 1e-3)
    return {"achieved": rate, "peak": peak, "unit": "wave64 VALU instructions/s",
            "frac": rate / peak, "instructions_per_pass": v["per_pass"],
            "instructions_per_segment": v["per_pass"] / v["segments_per_pass"],
            "source": "SQ_INSTS_VALU per pass from the committed counter summary over this "
                      "run's mean pass time; peak = 4 SIMDs x CUs x 2.4 GHz / 4 cycles"}


def valu_peak():
    """wave64 VALU instructions per second the device can issue: one per 4
    cycles on each SIMD (a 64-lane FP64 instruction occupies a 16-lane SIMD
    for 4 cycles), 4 SIMDs per CU."""
    import torch
    p = torch.cuda.get_device_properties(0)
    clock_hz = 2.4e9  # MI355X peak engine clock
    return 4 * p.multi_processor_count * clock_hz / 4.0


ATOMIC_PATTERNS = ("window", "scattered")


def atomic_peak(n_rounds=256):
    """The device's FP64 atomic-add rate (adds/s) in the two tally patterns
    (a wavefront's 64 consecutive doubles; a place per lane), on a table the
    size of the paper-scale J_blue array (20 x 3e5 doubles)."""
    import torch

    from paper_1401_5469_amd import smc

    table = torch.zeros(20 * 300_000, dtype=torch.float64, device="cuda")
    rates = {p: smc.measure_atomic_rate(table, n_rounds, scattered=(p == "scattered"))
             for p in ATOMIC_PATTERNS}
    del table
    return rates


def atomics(args):
    """Print the device's FP64 atomic-add rates in the tally patterns."""
    runs = [atomic_peak() for _ in range(3)]
    best = {p: max(r[p] for r in runs) for p in ATOMIC_PATTERNS}
    print(json.dumps({"metric": "FP64 atomic adds per second (tally patterns)",
                      "value": best["window"], "unit": "atomics/s", "by_pattern": best,
                      "runs": runs,
                      "pattern": "window: 64 consecutive doubles per wavefront at a "
                                 "pseudo-random place of a 48 MB table; scattered: a "
                                 "pseudo-random double per lane; 8 workgroups of 256 per CU, "
                                 "256 rounds, two launches each (the second timed)"}),
          flush=True)


def _kernel_name(k):
    k = k.replace("void ", "", 1).replace("smc::(anonymous namespace)::", "")
    return k.replace("smc::", "").split("(")[0]


def _pmc_dispatches(path):
    """Dispatches of a rocprofv3 --pmc database in order:
    [(kernel, grid size, duration ns, {counter: value})]."""
    import sqlite3

    con = sqlite3.connect(path)
    rows = con.execute("select dispatch_id, kernel_name, grid_size, duration, counter_name, value "
                       "from counters_collection order by dispatch_id").fetchall()
    out, index = [], {}
    for d, k, g, t, c, v in rows:
        if d not in index:
            index[d] = len(out)
            out.append((_kernel_name(k), int(g), float(t), {}))
        cs = out[index[d]][3]
        cs[c] = cs.get(c, 0.0) + float(v)
    return out


PASS_KERNELS = ("transport_kernel", "long_prefix_kernel", "order_count_kernel",
                "order_scan_kernel", "order_place_kernel", "long_kernel", "solo_kernel")


def _transport_passes(disp, warmup, steps):
    """The dispatches of the timed transport passes of a bench run: a pass
    opens at transport_kernel and holds the hand-off kernels after it; the
    first `warmup` passes are skipped, the next `steps` returned."""
    passes, cur = [], None
    for d in disp:
        base = d[0].split("<")[0]
        if base == "transport_kernel":
            cur = [d]
            passes.append(cur)
        elif base in PASS_KERNELS and cur is not None:
            cur.append(d)
        else:
            cur = None
    sel = passes[warmup:warmup + steps]
    if len(sel) != steps:
        raise SystemExit(f"found {len(passes)} transport passes, need {warmup + steps}")
    return sel


def _source_sha():
    import hashlib

    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _bench_line(path):
    with open(path) as f:
        lines = [l for l in f.read().splitlines() if l.startswith("{")]
    return json.loads(lines[-1])


def _algorithmic_bytes(line):
    """Algorithmic bytes per transport pass of a bench line (the byte model)."""
    return (BYTES_PER_LINE_PASS * line["line_passes_per_s"] + BYTES_PER_SEGMENT *
            line["segments_per_s"]) * line["ms_per_step"] * 1e-3 + \
        BYTES_PER_PACKET * line["config"]["packets_per_iteration"]


def traffic_summary(args):
    """HBM bytes per transport pass from FETCH_SIZE and WRITE_SIZE runs of
    the bench and of the 1 GiB device copy, which scales each counter to
    bytes.  Arguments: OUT BENCH_FETCH_DB BENCH_WRITE_DB COPY_FETCH_DB
    COPY_WRITE_DB BENCH_LINE (the bench's output of one of the runs)."""
    out, bf, bw, cf, cw, bl = args.traffic_summary
    n = 1 << 30
    copies = {}
    for name, db in (("FETCH_SIZE", cf), ("WRITE_SIZE", cw)):
        d = _pmc_dispatches(db)[-5:]  # the five timed copies end the run
        copies[name] = (sum(x[3][name] for x in d) / len(d), sorted({x[0] for x in d}))
    fetch_scale = n / (copies["FETCH_SIZE"][0] * 1024.0)
    write_scale = n / (copies["WRITE_SIZE"][0] * 1024.0)
    fp = _transport_passes(_pmc_dispatches(bf), args.warmup, args.steps)
    wp = _transport_passes(_pmc_dispatches(bw), args.warmup, args.steps)
    per = []
    for f, w in zip(fp, wp):
        fk = sum(d[3]["FETCH_SIZE"] for d in f)
        wk = sum(d[3]["WRITE_SIZE"] for d in w)
        per.append(1024.0 * (fetch_scale * fk + write_scale * wk))
    line = _bench_line(bl)
    alg = _algorithmic_bytes(line)
    summ = {
        "what": "HBM bytes per transport pass (transport_kernel, order kernels and the kernel "
                "of the handed-off histories) of the paper-scale scatter model, 1e6 packets "
                f"per iteration, mean over the {args.steps} timed iterations of a bench run "
                "(T_inner from 9000 K, carried on the device)",
        "commands": args.commands or [],
        "calibration": {"copy_bytes_read_and_written": n,
                        "FETCH_SIZE_KiB_per_copy": copies["FETCH_SIZE"][0],
                        "WRITE_SIZE_KiB_per_copy": copies["WRITE_SIZE"][0],
                        "copy_kernels": copies["FETCH_SIZE"][1],
                        "fetch_scale": fetch_scale, "write_scale": write_scale},
        "kernel_source_sha256": _source_sha(),
        "bytes_per_transport_pass": sum(per) / len(per),
        "bytes_per_transport_pass_by_iteration": per,
        "algorithmic_bytes_per_transport_pass": alg,
        "traffic_over_algorithmic": sum(per) / len(per) / alg,
    }
    with open(out, "w") as f:
        json.dump(summ, f, indent=1)
    print(json.dumps(summ, indent=1))


def counter_summary(args):
    """Per-pass and per-kernel hardware counters of the transport pass, from
    --pmc runs of the bench (any number of counter sets), with the atomic
    calibration from a --pmc run of --workload atomics.  Arguments: OUT
    BENCH_LINE ATOMICS_DB BENCH_DB [BENCH_DB ...]."""
    out, bl, adb, *dbs = args.counter_summary
    line = _bench_line(bl)
    per_pass, per_kernel, dur = {}, {}, {}
    for db in dbs:
        passes = _transport_passes(_pmc_dispatches(db), args.warmup, args.steps)
        for p in passes:
            for k, g, t, cs in p:
                fam = k.split("<")[0]
                dur.setdefault(db, []).append(t)
                for c, v in cs.items():
                    per_pass[c] = per_pass.get(c, 0.0) + v / len(passes)
                    kk = per_kernel.setdefault(fam, {})
                    kk[c] = kk.get(c, 0.0) + v / len(passes)
    segs = line["segments_per_s"] * line["ms_per_step"] * 1e-3
    # atomic calibration: grid x rounds adds per dispatch of atomic_rate_kernel
    cal = {}
    for k, g, t, cs in _pmc_dispatches(adb):
        if not k.startswith("atomic_rate_kernel"):
            continue
        pat = "scattered" if "<true>" in k else "window"
        adds = g * args.atomic_rounds
        e = cal.setdefault(pat, {"dispatches": 0, "adds": 0.0, "ns": 0.0, "counters": {}})
        e["dispatches"] += 1
        e["adds"] += adds
        e["ns"] += t
        for c, v in cs.items():
            e["counters"][c] = e["counters"].get(c, 0.0) + v
    calib = {}
    for pat, e in cal.items():
        calib[pat] = {"adds_per_dispatch": e["adds"] / e["dispatches"],
                      "dispatches": e["dispatches"],
                      "adds_per_s_under_counters": e["adds"] / (e["ns"] * 1e-9)}
        for c, v in e["counters"].items():
            calib[pat][c + "_per_add"] = v / e["adds"]
    summ = {
        "what": "hardware counters of the transport pass of the paper-scale scatter model "
                f"(1e6 packets per iteration), mean per pass over the {args.steps} timed "
                "iterations of a bench run, in total and per kernel; atomic counters of the "
                "FP64 atomic-add calibration kernel per add",
        "commands": args.commands or [],
        "kernel_source_sha256": _source_sha(),
        "segments_per_pass": segs,
        "per_pass": per_pass,
        "per_kernel": per_kernel,
        "per_segment": {c: v / segs for c, v in per_pass.items()},
        "atomic_calibration": calib,
    }
    with open(out, "w") as f:
        json.dump(summ, f, indent=1)
    print(json.dumps(summ, indent=1))


def trace_summary(args):
    """Kernel-trace summary of a rocprofv3 --kernel-trace --stats database:
    the top_kernels table, then per transport pass the durations of
    transport_kernel and of the kernel of the handed-off histories and the
    span from the first's start to the last pass kernel's end (the time the
    library's events bracket).  Arguments: DB [BENCH_LINE]."""
    import sqlite3

    db, *rest = args.trace_summary
    con = sqlite3.connect(db)
    print("name | calls | total_ms | average_ms | percent")
    for name, n, tot, avg, pct in con.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"):
        # this view holds microseconds, the kernels view nanoseconds
        print(f"{name} | {n} | {tot * 1e-3:.3f} | {avg * 1e-3:.3f} | {pct:.2f}")
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    print("\nper transport pass (ms): transport_kernel | hand-off kernels | handed-off "
          "histories kernel | span")
    cur = None
    passes = []
    for name, t0, t1 in rows:
        k = _kernel_name(name).split("<")[0]
        if k == "transport_kernel":
            cur = {"t0": t0, "t1": t1, "transport": t1 - t0, "order": 0, "long": 0, "kernel": ""}
            passes.append(cur)
        elif k in PASS_KERNELS and cur is not None:
            cur["t1"] = t1
            if k in ("long_kernel", "solo_kernel"):
                cur["long"] += t1 - t0
                cur["kernel"] = _kernel_name(name)
            else:
                cur["order"] += t1 - t0
        else:
            cur = None
    for p in passes:
        print(f"{p['transport'] * 1e-6:.3f} | {p['order'] * 1e-6:.3f} | "
              f"{p['long'] * 1e-6:.3f} ({p['kernel']}) | {(p['t1'] - p['t0']) * 1e-6:.3f}")
    if rest:
        line = _bench_line(rest[0])
        print("\nthe same run's bench line: transport_ms (library HIP events) = " +
              ", ".join(f"{t:.3f}" for t in line["transport_ms"]))
        print(f"interactions/s over the timed iterations: {line['value']:.4g}")


def profile_summary(paths, last=0, kernel=""):
    """Per-kernel sums of the counters in rocprofv3 --pmc result databases,
    with the dispatch count and mean duration (one table per database)."""
    from collections import defaultdict

    for path in paths:
        per = defaultdict(lambda: defaultdict(float))
        n = defaultdict(int)
        dur = defaultdict(float)
        for k, g, t, cs in _pmc_dispatches(path):
            n[k] += 1
            dur[k] += t
            for c, v in cs.items():
                per[k][c] += v
        print(f"# {os.path.basename(os.path.dirname(path))}")
        for name in sorted(per, key=lambda k: -dur[k]):
            cs = "  ".join(f"{c}={v:.6g}" for c, v in sorted(per[name].items()))
            print(f"{name} | dispatches {n[name]} | mean {dur[name] / n[name] * 1e-6:.3f} ms | {cs}")
        if last:
            sel = [d for d in _pmc_dispatches(path) if kernel in d[0]][-last:]
            print(f"# the last {last} dispatches" + (f" of {kernel}" if kernel else ""))
            for k, g, t, cs in sel:
                c = "  ".join(f"{c}={v:.6g}" for c, v in sorted(cs.items()))
                print(f"{k} | grid {g} | {t * 1e-6:.3f} ms | {c}")


def copy_reference(args):
    """Plain device copies of 1 GiB: what the HBM byte counters read for a
    kernel that moves a known number of bytes."""
    import torch

    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"metric": "device copy bandwidth", "value": 2 * n / dt / 1e9,
                      "unit": "GB/s", "bytes_read_per_copy": n, "bytes_written_per_copy": n,
                      "copies": 5}), flush=True)


def virtual(args):
    """The paper-scale model: the iterative sequence (T_inner carried on the
    device) without virtual packets, then the final spectrum iteration once
    plain and once with N_v virtual packets per packet launch (section 2.9).
    Reports the cost of the v-packet iteration and its v-packet rates."""
    import numpy as np
    import torch

    from paper_1401_5469_amd import smc
    from paper_1401_5469_amd import workloads as W

    w = W.config2(n_packets=args.packets)
    N = w.n_packets
    flags = 0 if args.no_jblue else smc.F_JBLUE
    ctx = smc.Context(0)
    model = smc.Model(ctx, w.model, N, flags=flags)
    for i in range(args.steps):
        model.run_iteration(N, w.T_inner if i == 0 else 0.0, iteration=i, flags=flags,
                            L_requested=w.L_requested, damping=w.damping)
    torch.cuda.synchronize()
    T_final = model.read_spectrum()["T_inner_next"]
    print(f"# {args.steps} iterations, T_inner -> {T_final:.1f} K", file=sys.stderr, flush=True)
    out_runs = {}
    for nv in (0, args.n_virtual):
        t0 = time.perf_counter()
        model.run_iteration(N, T_final, iteration=args.steps, flags=flags | smc.F_TIMING,
                            n_virtual=nv)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rec = dict(wall_ms=wall * 1e3, transport_ms=model.read_timing(),
                   counters=model.read_counters())
        if nv:
            vs = model.read_virtual_spectrum()
            rec.update(v_counts=vs["counts"], L_virtual=vs["L_total"],
                       L_emitted=model.read_spectrum()["L_emitted"])
        out_runs[nv] = rec
        print(f"# final iteration with n_virtual={nv}: {wall * 1e3:.1f} ms", file=sys.stderr,
              flush=True)
    v = out_runs[args.n_virtual]
    wall = v["wall_ms"] * 1e-3
    out = {
        "metric": "virtual packets/sec (final spectrum iteration)",
        "value": v["v_counts"]["launched"] / wall,
        "unit": "v-packets/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": args.steps,
        "ms_per_step": v["wall_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}-final-spectrum-nv{args.n_virtual}",
                   "packets": N, "n_virtual": args.n_virtual, "T_inner": T_final},
        "virtual": {"v_packets_launched": v["v_counts"]["launched"],
                    "v_packets_counted": v["v_counts"]["counted"],
                    "v_line_resonances": v["v_counts"]["passes"],
                    "v_line_resonances_per_s": v["v_counts"]["passes"] / wall,
                    "L_virtual": v["L_virtual"], "L_emitted": v["L_emitted"]},
        "plain_final_iteration_ms": out_runs[0]["wall_ms"],
        "cost_ratio": v["wall_ms"] / out_runs[0]["wall_ms"],
    }
    print(json.dumps(out), flush=True)


def macroatom(args):
    """One iteration of 5e5 packets through the 30-shell model in macroatom
    mode (8 elements x 5 stages x 40 levels, 2e4 lines; tau_S, n_e and the
    per-shell transition tables from the plasma state of the initial field,
    nebular / dilute-LTE), and through the same model in downbranch form:
    the same tables with every internal jump removed and each row
    renormalised over its deactivations (Table 1: the macro atom with its
    internal probabilities set to zero), so that the two runs differ only by
    the jumps.  Reports interactions/s of both and the cost ratio (the paper
    quotes about +10% for macroatom over downbranch), and the time of the
    plasma update that derives the tables."""
    import numpy as np
    import torch

    from paper_1401_5469_amd import smc
    from paper_1401_5469_amd import workloads as W

    ctx = smc.Context(0)
    w, spec = W.config_macroatom()
    N = w.n_packets
    ma = smc.Model(ctx, w.model, N, flags=smc.F_JBLUE)
    pl = smc.Plasma(ma, spec)
    pl.update(W.ION_NEBULAR, W.EXC_DILUTE_LTE)
    torch.cuda.synchronize()
    ups = []
    for _ in range(5):
        t0 = time.perf_counter()
        pl.update(W.ION_NEBULAR, W.EXC_DILUTE_LTE)
        torch.cuda.synchronize()
        ups.append(time.perf_counter() - t0)
    # the downbranch form of the same tables
    ptr, line, cum = ma.read_macroatom()
    st = pl.read(level_pop=False)
    db_cum = np.empty_like(cum)
    for lev in range(len(ptr) - 1):
        a, b = int(ptr[lev]), int(ptr[lev + 1])
        if b == a:
            continue
        p = np.diff(np.concatenate([np.zeros((cum.shape[0], 1)), cum[:, a:b]], axis=1), axis=1)
        p[:, line[a:b] < 0] = 0.0
        run = np.cumsum(p, axis=1)  # sequential: never above its last entry
        tot = run[:, -1:]
        c = np.where(tot > 0, run / np.where(tot > 0, tot, 1.0), 1.0)
        c[:, -1] = 1.0
        db_cum[:, a:b] = c
    db_model = W.Model(**{**w.model.__dict__, "tau_sobolev": np.ascontiguousarray(st["tau"]),
                          "n_e": np.ascontiguousarray(st["n_e"]), "level_ptr": ptr,
                          "em_line": line, "em_cum": np.ascontiguousarray(db_cum)})
    db = smc.Model(ctx, db_model, N, flags=smc.F_JBLUE)
    res = {}
    for name, model in (("macroatom", ma), ("downbranch", db)):
        for _ in range(args.warmup):
            model.run_iteration(N, w.T_inner, flags=smc.F_JBLUE)
        torch.cuda.synchronize()
        walls, inter = [], []
        for i in range(args.steps):
            t0 = time.perf_counter()
            model.run_iteration(N, w.T_inner, iteration=i, flags=smc.F_JBLUE)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            c = model.read_counters()
            inter.append(c["line_events"] + c["escatters"])
        wall = float(np.mean(walls))
        res[name] = dict(workload=w.name, packets=N, ms=wall * 1e3,
                         interactions_per_s=float(np.mean(inter)) / wall,
                         packets_per_s=N / wall, counters=c)
        print(f"# {name}: {wall * 1e3:.2f} ms per iteration", file=sys.stderr, flush=True)
    del pl
    r_ma = res["macroatom"]
    out = {
        "metric": "packet-interactions/sec (macroatom mode)",
        "value": r_ma["interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r_ma["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": r_ma["workload"], "packets": N, "shells": w.model.n_shells,
                   "lines": w.model.n_lines, "levels": int(w.model.n_levels),
                   "tables": "derived on the device from the plasma state"},
        "macroatom": r_ma,
        "downbranch": res["downbranch"],
        "ms_ratio_macroatom_over_downbranch": r_ma["ms"] / res["downbranch"]["ms"],
        "interaction_cost_ratio": res["downbranch"]["interactions_per_s"] /
        r_ma["interactions_per_s"],
        "plasma_update_with_tables_ms": 1e3 * min(ups),
    }
    print(json.dumps(out), flush=True)


def plasma(args):
    """Iterations of the paper-scale plasma model (20 shells, 3e5 lines of 8
    synthetic elements x 5 stages x 150 levels, 1e6 packets): after every
    iteration the plasma update (nebular ionization, dilute-LTE excitation)
    rewrites tau_S and n_e from the iteration's T_R and W; T_inner moves
    toward the requested luminosity after every third iteration (the scheme
    of section 5.3).  The first timed iteration starts again from T_inner =
    9000 K and the opacities of the initial field.  The value is
    interactions per second over the whole loop, plasma updates included;
    the roofline entry prices the plasma update (state and depth kernels,
    timed together with HIP events on the launch stream) at its algorithmic
    bytes: tau_S written once, the per-line records and the level
    populations read once, the atomic data and densities read per shell.
    With --nlte the stage-1 ions of the Mg, Si, S and Ca analogues (40
    levels each) take their populations from statistical equilibrium, with
    J_b from the J_blue estimator of the iteration before (W B_nu(T_R) before
    the first) and escape probabilities from the depths in the model."""
    import numpy as np
    import torch

    from oracle import plasma as OP
    from paper_1401_5469_amd import smc
    from paper_1401_5469_amd import workloads as W

    nlte = bool(args.nlte)
    w, spec = (W.config_plasma_nlte if nlte else W.config_plasma)(n_packets=args.packets)
    m_in, a = w.model, spec.atom
    N, S, L = w.n_packets, m_in.n_shells, m_in.n_lines
    ion, exc = W.ION_NEBULAR, W.EXC_DILUTE_LTE
    flags = 0 if args.no_jblue else smc.F_JBLUE
    jb = smc.JB_DETAILED if (nlte and flags) else smc.JB_DILUTE_BLACKBODY
    ctx = smc.Context(0)
    model = smc.Model(ctx, m_in, N, flags=flags)
    pl = smc.Plasma(model, spec)
    v = m_in.v_bounds
    q = v[0] / (0.5 * (v[:-1] + v[1:]))
    T0, W0 = np.full(S, 1.0e4), 0.5 * (1.0 - np.sqrt(1.0 - q * q))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run(k, record):
        pl.update(ion, exc, T_R=T0, W=W0, nlte=nlte)
        for i in range(k):
            model.run_iteration(N, w.T_inner if i == 0 else 0.0, iteration=i,
                                flags=flags | smc.F_TIMING,
                                L_requested=w.L_requested if i % 3 == 2 else 0.0,
                                damping=w.damping)
            ev0.record()
            pl.update(ion, exc, nlte=nlte, jblue_mode=jb)
            ev1.record()
            c = model.read_counters()
            ms = model.read_timing()
            ev1.synchronize()
            pms = ev0.elapsed_time(ev1)
            s = model.read_spectrum()
            if record is not None:
                record.append((c, ms, pms, s["T_inner"]))
            print(f"# iteration {i}: {ms:.2f} ms transport, {pms:.3f} ms plasma update, "
                  f"T_inner {s['T_inner']:.0f} K", file=sys.stderr, flush=True)

    run(args.warmup, None)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    run(args.steps, rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = pl.read(tau=False, level_pop=False)

    inter = sum(c["line_events"] + c["escatters"] for c, _, _, _ in rec)
    pms = [p for _, _, p, _ in rec]
    mean_pms = float(np.mean(pms))
    NI, NL, E = a.n_ions, a.n_levels, a.n_elements
    # tau_S written; 16-byte line records read; n and n / g written, n / g
    # read back; level data (energy, g, flag, ion) read; ion densities and
    # partition functions written; element densities read
    bytes_update = (S * L * 8 + L * 16 + S * NL * 8 * 3 + NL * (8 + 8 + 1 + 4)
                    + S * NI * 8 * 2 + S * E * 8)
    n_nlte_lines = 0
    for i in spec.nlte_ions if nlte else ():
        l0, l1 = a.ion_level_ptr[i], a.ion_level_ptr[i + 1]
        n_nlte_lines += int(((a.line_lower >= l0) & (a.line_lower < l1)).sum())
    # NLTE: per line a 64-byte record, tau_S and J_blue read in every shell
    bytes_update += n_nlte_lines * 64 + S * n_nlte_lines * 16
    achieved = bytes_update / (mean_pms * 1e-3) / 1e9
    # the plasma oracle on the same inputs (numpy FP64, one update)
    t1 = time.perf_counter()
    OP.plasma_state(a, spec.number_density, m_in.line_nu, m_in.t_exp, T0, W0, ion, exc,
                    nlte_ions=spec.nlte_ions if nlte else ())
    cpu_s = time.perf_counter() - t1
    out = {
        "metric": "packet-interactions/sec (with plasma feedback"
                  + (", NLTE)" if nlte else ")"),
        "value": inter / wall,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "shells": S, "lines": L, "elements": E, "ions": NI,
                   "levels": NL, "packets_per_iteration": N, "ionization": "nebular",
                   "excitation": "dilute-lte", "T_inner_start": w.T_inner,
                   "nlte_ions": list(spec.nlte_ions) if nlte else [],
                   "jblue_mode": "detailed" if jb == smc.JB_DETAILED else "dilute-blackbody"},
        "transport_ms": [m for _, m, _, _ in rec],
        "plasma_update_ms": pms,
        "T_inner": [t for _, _, _, t in rec],
        "n_e_final": st["n_e"].tolist(),
        "inverted_lines_final": st["n_clamped"],
        "singular_nlte_systems_final": st["n_singular"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "plasma update: plasma_state_kernel + "
                               + ("plasma_nlte_kernel + " if nlte else "") + "plasma_tau_kernel",
                     "bytes_per_launch": bytes_update},
        "cpu_baseline": {"value": 1.0 / cpu_s, "unit": "plasma updates/s", "cores": 1,
                         "kind": "oracle",
                         "sample": f"one plasma update of the whole model on the initial field "
                                   f"({S} shells x {L} lines"
                                   + (f", {len(spec.nlte_ions)} NLTE ions" if nlte else "")
                                   + f", numpy FP64, {cpu_s:.2f} s)"},
        "plasma_updates_per_s": 1e3 / mean_pms,
    }
    print(json.dumps(out), flush=True)


def _oracle_jobs(w, jobs):
    """The oracle on jobs [(iteration, T_inner, lo, hi), ...]: packet ids
    [lo, hi) of each iteration at its T_inner.  Summed counters and seconds."""
    from oracle import oracle as O
    import numpy as np

    tot, dt = None, 0.0
    for it, T, lo, hi in jobs:
        if hi <= lo:
            continue
        ids = np.arange(lo, hi, dtype=np.uint64)
        t0 = time.perf_counter()
        r = O.run(w.model, T, w.n_packets, iteration=it, packet_ids=ids, want_jblue=True,
                  want_packets=False)
        dt += time.perf_counter() - t0
        c = r["counters"]
        tot = dict(c) if tot is None else {k: tot[k] + c[k] for k in tot}
    return tot, dt


def cpu_worker(args):
    """One process of the all-cores baseline: no GPU, one JSON line."""
    from paper_1401_5469_amd import workloads as W

    w = W.config2(n_packets=args.packets)
    c, dt = _oracle_jobs(w, json.loads(args.cpu_worker))
    print(json.dumps({"counters": c, "seconds": dt}), flush=True)


def cpu_baseline(w, n_sample, procs, schedule):
    """The FP64 oracle on a sample of the timed iterations: `schedule` lists
    the (iteration, T_inner) of each, and each contributes packet ids
    0..n_sample/len(schedule)-1.  Run once in this process on one core, then
    with every iteration's ids split into `procs` disjoint ranges run by as
    many oracle processes at once (wall time = the slowest)."""
    import subprocess
    from oracle import build as ob

    if not os.path.exists(ob.LIB):
        ob.build()
    per = max(1, n_sample // len(schedule))
    jobs = [(it, T, 0, per) for it, T in schedule]
    c, dt = _oracle_jobs(w, jobs)
    inter = c["line_events"] + c["escatters"]
    single = {"value": inter / dt, "unit": "interactions/s", "cores": 1, "seconds": dt,
              "packets_per_s": per * len(jobs) / dt, "segments_per_s": c["segments"] / dt,
              "line_passes_per_s": c["line_passes"] / dt}
    edges = [per * k // procs for k in range(procs + 1)]
    parts = [[(it, T, a, b) for it, T in schedule] for a, b in zip(edges[:-1], edges[1:])
             if b > a]
    workers = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--packets",
                                 str(w.n_packets), "--cpu-worker", json.dumps(p)],
                                stdout=subprocess.PIPE, text=True) for p in parts]
    res = []
    for p in workers:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed with status {p.returncode}")
        res.append(json.loads(out.strip().splitlines()[-1]))
    wall = max(r["seconds"] for r in res)
    tot = {k: sum(r["counters"][k] for r in res) for k in res[0]["counters"]}
    inter_all = tot["line_events"] + tot["escatters"]
    assert inter_all == inter, "the split sample must hold the same interactions"
    temps = ", ".join(f"{T:.0f}" for _, T in schedule)
    return {"value": inter_all / wall, "unit": "interactions/s", "cores": len(workers),
            "kind": "oracle",
            "sample": f"packet ids 0..{per - 1} of each timed iteration "
                      f"{schedule[0][0]}..{schedule[-1][0]} at the T_inner the device used "
                      f"({temps} K): {inter} interactions, {c['segments']} segments, split "
                      f"over {len(workers)} single-threaded FP64 C oracle processes on "
                      f"disjoint id ranges (slowest {wall:.2f} s); the same sample in one "
                      f"process took {dt:.2f} s",
            "packets_per_s": per * len(jobs) / wall, "segments_per_s": tot["segments"] / wall,
            "line_passes_per_s": tot["line_passes"] / wall, "seconds": wall,
            "interactions_per_packet": inter / (per * len(jobs)),
            "single_core": single}


def batched_measure(n_models, steps, warmup, jblue, log=True):
    """64 models of uneven size (shells U{10..100}, lines log-uniform 1e4-3e5,
    packets log-uniform 1e5-1e6, otherwise as the paper-scale model; model i
    from seed i), one iteration each: one autotuned multi-model launch per
    step against the 64 single-model launches one after the other, with the
    same packets.  Returns the measurement (models/s of both forms)."""
    import numpy as np
    import torch

    from paper_1401_5469_amd import smc
    from paper_1401_5469_amd import workloads as W

    t0 = time.perf_counter()
    mix = [W.config4_model(i) for i in range(n_models)]
    gen_s = time.perf_counter() - t0
    flags = smc.F_JBLUE if jblue else 0
    ctx = smc.Context(0)
    models = [smc.Model(ctx, w.model, w.n_packets, flags=flags) for w in mix]
    torch.cuda.synchronize()
    if log:
        print(f"# {len(mix)} models generated in {gen_s:.1f} s and loaded", file=sys.stderr,
              flush=True)
    params = [dict(n_packets=w.n_packets, T_inner=w.T_inner, iteration=0, flags=flags)
              for w in mix]

    def counts(ms):
        c = [m.read_counters() for m in ms]
        return (sum(x["line_events"] + x["escatters"] for x in c), sum(x["segments"] for x in c))

    # plain form: one single-model iteration after the other
    for m, p in zip(models[:2], params[:2]):
        m.run_iteration(**p)  # warm-up
    torch.cuda.synchronize()
    plain_walls = []
    for step in range(steps):
        t0 = time.perf_counter()
        for m, p in zip(models, params):
            m.run_iteration(**p)
        torch.cuda.synchronize()
        plain_walls.append(time.perf_counter() - t0)
        if log:
            print(f"# plain step {step}: {plain_walls[-1] * 1e3:.1f} ms", file=sys.stderr,
                  flush=True)
    inter, segs = counts(models)

    # batched form with the library's default tuning
    ctx.batch_run(models, params)
    torch.cuda.synchronize()
    dwalls = []
    for step in range(steps):
        t0 = time.perf_counter()
        ctx.batch_run(models, params)
        torch.cuda.synchronize()
        dwalls.append(time.perf_counter() - t0)
    if log:
        print(f"# batched, default tuning: {np.mean(dwalls) * 1e3:.1f} ms", file=sys.stderr,
              flush=True)

    # batched form: the autotuned multi-model launch
    t0 = time.perf_counter()
    best, best_ms = ctx.batch_autotune(models, params)
    tune_s = time.perf_counter() - t0
    if log:
        print(f"# autotune: {best} {best_ms:.1f} ms ({tune_s:.1f} s)", file=sys.stderr, flush=True)
    for _ in range(warmup):
        ctx.batch_run(models, params, tune=best)
    torch.cuda.synchronize()
    walls, kern = [], []
    for step in range(steps):
        t0 = time.perf_counter()
        ctx.batch_run(models, params, tune=best, timing=True)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        kern.append(ctx.batch_read_timing())
        if log:
            print(f"# batched step {step}: {walls[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    b_inter, b_segs = counts(models)
    n = len(mix)
    wall = float(np.mean(walls))
    plain = float(np.mean(plain_walls))
    out = {
        "workload": f"batched-{n}-models", "models": n, "steps": steps,
        "packets_total": int(sum(w.n_packets for w in mix)),
        "shells_mean": float(np.mean([w.model.n_shells for w in mix])),
        "lines_mean": float(np.mean([w.model.n_lines for w in mix])),
        "batched": {"models_per_s": n / wall, "interactions_per_s": b_inter / wall,
                    "segments_per_s": b_segs / wall, "wall_ms": wall * 1e3,
                    "transport_ms": kern, "tune": best,
                    "autotune_s": tune_s, "autotune_note": "coordinate search, two timed runs "
                    "per candidate, a candidate kept only when 2 % faster; not in wall_ms"},
        "batched_default_tune": {"models_per_s": n / float(np.mean(dwalls)),
                                 "wall_ms": float(np.mean(dwalls)) * 1e3},
        "plain": {"models_per_s": n / plain, "interactions_per_s": inter / plain,
                  "segments_per_s": segs / plain, "wall_ms": plain * 1e3},
        "speedup_vs_plain": plain / wall,
        "interactions_per_step": b_inter,
    }
    for m in models:
        m.free()
    ctx.close()
    return out


def batched(args):
    """The batched mix as its own bench line (value: models/s batched)."""
    r = batched_measure(args.models, args.steps, args.warmup, not args.no_jblue)
    out = {
        "metric": "models/sec (batched)",
        "value": r["batched"]["models_per_s"],
        "unit": "models/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["batched"]["wall_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": r["workload"], "models": r["models"],
                   "packets_total": r["packets_total"], "shells_mean": r["shells_mean"],
                   "lines_mean": r["lines_mean"], "jblue": not args.no_jblue},
        "batched": r["batched"],
        "plain": r["plain"],
        "speedup_vs_plain": r["speedup_vs_plain"],
        "interactions_per_step": r["interactions_per_step"],
    }
    print(json.dumps(out), flush=True)


def _gen_request(args):
    t, seed, n_iter = args
    from paper_1401_5469_amd import workloads as W
    w = W.config4_model(seed)
    return t, seed, n_iter, w


class _Feed:
    """Request models built in worker processes ahead of their arrival: at
    most `window` in flight or waiting, so that host memory holds a few GB
    rather than the whole arrival list."""

    def __init__(self, pool, arrivals, window=64):
        self.pool, self.arrivals, self.window = pool, arrivals, window
        self.jobs = {}
        self.next = 0
        for _ in range(min(window, len(arrivals))):
            self._queue()

    def _queue(self):
        if self.next < len(self.arrivals):
            self.jobs[self.next] = self.pool.apply_async(_gen_request, (self.arrivals[self.next],))
            self.next += 1

    def get(self, j):
        out = self.jobs.pop(j).get()
        self._queue()
        return out


def _request(serve, g):
    t, seed, n_iter, w = g
    return serve.Request(model=w.model, n_iterations=n_iter, n_packets=w.n_packets,
                         T_inner=w.T_inner, L_requested=w.L_requested, damping=w.damping,
                         arrival=t)


def _serve_mode(mode, serve, be, pool, arrivals, budget, n_streams, max_active, max_cohort,
                log):
    """Drive one server over the arrival list in real time, submitting each
    request when it arrives (its model built ahead by the pool).  Returns the
    server's statistics, its wall time and the requests."""
    feed = _Feed(pool, arrivals)
    srv = (serve.StreamServer(be, memory_budget=budget, n_streams=n_streams,
                              max_active=max_active, max_cohort=max_cohort) if mode == "stream"
           else serve.Server(be, memory_budget=budget, max_active=max_active))
    reqs = []
    n, j, last, k_adm = len(arrivals), 0, 0, 0
    t0 = time.perf_counter()
    while j < n or srv.pending or srv.active:
        while j < n and arrivals[j][0] <= srv.now():
            r = _request(serve, feed.get(j))
            srv.submit(r)
            reqs.append(r)
            j += 1
        moved = srv.advance() if mode == "stream" else srv.step()
        if not moved:
            nxt = arrivals[j][0] - srv.now() if j < n else None
            busy = mode == "stream" and srv.busy()
            if busy:
                time.sleep(0.0005 if nxt is None else max(0.0, min(0.0005, nxt)))
            elif nxt is not None:
                time.sleep(max(0.0, nxt))
        # admission is in arrival order: the host copies of admitted models
        # are no longer needed
        while k_adm < len(reqs) and reqs[k_adm].state != serve.QUEUED:
            reqs[k_adm].model = None
            k_adm += 1
        done = len(reqs) - len(srv.active) - len(srv.pending)
        if done >= last + 100:
            last = done
            log(f"# {mode}: served {done}/{n} at {srv.now():.1f} s, active {len(srv.active)}")
    wall = time.perf_counter() - t0
    for r in reqs:
        r.model = None
    return srv.stats(), wall, reqs


def _compare_results(a, b):
    """Requests served two ways: counters equal, and the largest relative
    difference of J, nu-bar, T_R, W, L_nu, L_emitted and T_inner."""
    import numpy as np

    worst, same = 0.0, 0
    for x, y in zip(a, b):
        rx, ry = x.result, y.result
        same += rx["counters"] == ry["counters"]
        for k in ("J", "nubar", "T_R", "W", "L_nu"):
            u, v = np.asarray(rx[k]), np.asarray(ry[k])
            den = np.maximum(np.abs(v), 1e-300)
            worst = max(worst, float(np.max(np.abs(u - v) / den)) if u.size else 0.0)
        for k in ("T_inner", "T_inner_next", "L_emitted"):
            if rx[k] is not None and ry[k]:
                worst = max(worst, abs(rx[k] - ry[k]) / abs(ry[k]))
    return {"requests": len(a), "counters_equal": same, "max_rel_diff": worst}


def served(args):
    """Poisson arrivals at 20 requests/s for --duration seconds; request j is
    a model drawn as in the batched mix from seed 1000+j with U{1..10}
    iterations (every model kept resident on the device between its
    iterations, admitted while its workspace fits the memory budget).  Three
    paths over the same requests: the stream server (no global step:
    cohorts launched concurrently on --streams streams, a new arrival waits
    only for a free stream), the step-synchronous server (one multi-model
    launch per step for every admitted request, waited for), and the plain
    path (one request at a time, one single-model launch per iteration) on
    the first --plain-requests requests, whose plain latencies do not depend
    on later arrivals.  Reports latency, queue wait (arrival to first launch)
    and service time (first launch to completion), models/s, and whether
    every served result equals the plain path's (counters, and estimators to
    rounding)."""
    import multiprocessing as mp

    from paper_1401_5469_amd import serve
    from paper_1401_5469_amd import workloads as W

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    arrivals = W.config5_requests(duration_s=args.duration)
    modes = [m for m in args.served_modes.split(",") if m]
    # the model builders fork before anything touches the GPU
    pool = mp.get_context("fork").Pool(min(16, os.cpu_count() or 1))
    budget = int(args.budget_gb * 2**30)
    be = serve.GpuBackend(flags=None, keep_jblue=False)
    res, reqs_of = {}, {}
    for mode in modes:
        if mode == "plain":
            k = min(args.plain_requests, len(arrivals))
            feed = _Feed(pool, arrivals[:k])
            reqs = [None] * k

            def ordered():
                for j in range(k):
                    reqs[j] = _request(serve, feed.get(j))
                    yield reqs[j]
                    reqs[j].model = None
            t0 = time.perf_counter()
            st = serve.serve_plain(be, ordered(), ordered=True)
            wall = time.perf_counter() - t0
            st["requests"] = k
        else:
            st, wall, reqs = _serve_mode(mode, serve, be, pool, arrivals, budget, args.streams,
                                         args.max_active, args.max_cohort, log)
        packets = sum(r.n_packets * r.n_iterations for r in reqs)
        st.update(wall_s=wall, packets_per_s=packets / wall)
        res[mode] = st
        reqs_of[mode] = reqs
        log(f"# {mode}: {json.dumps(st)}")
    pool.close()
    out = {
        "metric": "p99 synthesis latency (served)",
        "value": res[modes[0]]["p99_s"] if modes[0] != "plain" else None,
        "unit": "s",
        "n_gpus": 1,
        "steps": res[modes[0]].get("steps"),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"served-poisson-20hz-{args.duration:g}s", "requests": len(arrivals),
                   "iterations_total": int(sum(n for _, _, n in arrivals)),
                   "budget_gb": args.budget_gb, "streams": args.streams,
                   "max_active": args.max_active, "max_cohort": args.max_cohort,
                   "server": modes[0]},
        **{m: res[m] for m in modes},
        "result_checks": {},
    }
    if "plain" in reqs_of:
        k = len(reqs_of["plain"])
        for m in modes:
            if m != "plain":
                byarr = sorted(reqs_of[m], key=lambda r: r.arrival)[:k]
                out["result_checks"][f"{m}_vs_plain"] = _compare_results(byarr, reqs_of["plain"])
                # the same first k requests as served
                out[m]["first_k"] = serve.latency_stats(byarr)
    if "stream" in res and "step" in res:
        out["stream_over_step"] = {
            "p50": res["step"]["p50_s"] / res["stream"]["p50_s"],
            "p99": res["step"]["p99_s"] / res["stream"]["p99_s"],
            "models_per_s": res["stream"]["models_per_s"] / res["step"]["models_per_s"]}
    print(json.dumps(out), flush=True)


def host_boundary(ctx, w, flags, N, interactions, wall, steps):
    """The same job with the host side of the boundary counted (untimed
    for `value`): the model handed over from host arrays (validation and
    upload of the line list and the Sobolev-depth table), and after every
    iteration the estimators, J_blue included, and the spectrum copied back
    to host memory."""
    import torch

    from paper_1401_5469_amd import smc

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = smc.Model(ctx, w.model, N, flags=flags)
    torch.cuda.synchronize()
    load = time.perf_counter() - t0
    m.run_iteration(N, w.T_inner, iteration=0, flags=flags, L_requested=w.L_requested,
                    damping=w.damping)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.read_estimators(jblue=bool(flags & smc.F_JBLUE))
    m.read_spectrum()
    read = time.perf_counter() - t0
    total = wall + load + steps * read
    return {"value": interactions / total, "unit": "interactions/s", "load_s": load,
            "read_s_per_iteration": read, "seconds": total}


def critical_path(ctx, w, flags, iteration, T_inner, pass_ms):
    """Latency bound of one transport pass: the longest history of the last
    timed iteration, found in a replay of that iteration with per-packet
    records, then run alone (a one-id launch, best of 3).  Histories depend
    only on (seed, iteration, packet id, T_inner), so the replay and the lone
    run follow the timed pass's history exactly; no pass can end before its
    longest history, which runs segment after segment."""
    import numpy as np

    from paper_1401_5469_amd import smc

    N = w.n_packets
    pm = smc.Model(ctx, w.model, N, flags=flags | smc.F_PACKETS)
    pm.run_iteration(N, T_inner, iteration=iteration, flags=flags | smc.F_PACKETS,
                     L_requested=w.L_requested, damping=w.damping)
    g = pm.read_packets(N)
    k = int(np.argmax(g["n_segments"]))
    pid, n_seg = int(g["id"][k]), int(g["n_segments"][k])
    alone = []
    for _ in range(3):
        pm.run_iteration(N, T_inner, iteration=iteration, flags=flags | smc.F_TIMING,
                         L_requested=w.L_requested, damping=w.damping,
                         packet_ids=np.array([pid], dtype=np.uint64))
        alone.append(pm.read_timing())
    a = min(alone)
    return {"packet_id": pid, "T_inner": T_inner, "iteration": iteration, "segments": n_seg,
            "alone_ms": a, "us_per_segment_alone": a * 1e3 / n_seg, "pass_ms": pass_ms,
            "frac": a / pass_ms}


def critical(args):
    """The latency bound alone: the iterative sequence from T_inner = 9000 K
    for --steps iterations, then the longest history of the last one run
    alone (critical_path; for counter runs of the lone history)."""
    import torch

    from paper_1401_5469_amd import smc
    from paper_1401_5469_amd import workloads as W

    w = W.config2(n_packets=args.packets)
    N = w.n_packets
    flags = 0 if args.no_jblue else smc.F_JBLUE
    ctx = smc.Context(0)
    model = smc.Model(ctx, w.model, N, flags=flags)
    for i in range(args.steps):
        model.run_iteration(N, w.T_inner if i == 0 else 0.0, iteration=i,
                            flags=flags | smc.F_TIMING, L_requested=w.L_requested,
                            damping=w.damping)
    ms = model.read_timing()
    T = model.read_spectrum()["T_inner"]
    model.free()
    torch.cuda.synchronize()
    out = critical_path(ctx, w, flags, args.steps - 1, T, ms)
    print(json.dumps({"metric": "critical-path microseconds per segment",
                      "value": out["us_per_segment_alone"], "unit": "us/segment",
                      "higher_is_better": False, "critical_path": out}), flush=True)


def main():
    args = parse()
    if args.profile_summary:
        return profile_summary(args.profile_summary, args.profile_last, args.profile_kernel)
    if args.traffic_summary:
        return traffic_summary(args)
    if args.counter_summary:
        return counter_summary(args)
    if args.trace_summary:
        return trace_summary(args)
    if args.cpu_worker:
        return cpu_worker(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (across GPUs "
              "the transport would shard by packet ids, one replica of the model per GPU, "
              "with one all-reduce of the tallies per iteration)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        if args.steps == 10:
            args.steps = 3
        return batched(args)
    if args.workload == "served":
        return served(args)
    if args.workload == "copy":
        return copy_reference(args)
    if args.workload == "virtual":
        return virtual(args)
    if args.workload == "macroatom":
        if args.steps == 10:
            args.steps = 3
        return macroatom(args)
    if args.workload == "plasma":
        return plasma(args)
    if args.workload == "atomics":
        return atomics(args)
    if args.workload == "critical":
        return critical(args)

    import numpy as np
    import torch

    from paper_1401_5469_amd import smc
    from paper_1401_5469_amd import workloads as W

    w = W.config2(n_packets=args.packets)
    N = w.n_packets
    flags = (0 if args.no_jblue else smc.F_JBLUE)
    ctx = smc.Context(0)
    model = smc.Model(ctx, w.model, N, flags=flags)
    torch.cuda.synchronize()

    def run(k, record):
        for i in range(k):
            model.run_iteration(N, w.T_inner if i == 0 else 0.0, iteration=i,
                                flags=flags | smc.F_TIMING, L_requested=w.L_requested,
                                damping=w.damping)
            c = model.read_counters()
            ms = model.read_timing()
            if record is not None:
                s = model.read_spectrum()
                record.append((c, ms, s["T_inner"], s["L_emitted"] / s["L_inner"]))
            print(f"# iteration {i}: {ms:.2f} ms transport, "
                  f"{c['line_events'] + c['escatters']} interactions", file=sys.stderr,
                  flush=True)

    run(args.warmup, None)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    run(args.steps, rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    inter = sum(c["line_events"] + c["escatters"] for c, _, _, _ in rec)
    segs = sum(c["segments"] for c, _, _, _ in rec)
    passes = sum(c["line_passes"] for c, _, _, _ in rec)
    kern_ms = [ms for _, ms, _, _ in rec]
    mean_ms = float(np.mean(kern_ms))
    bytes_per_launch = (BYTES_PER_LINE_PASS * passes + BYTES_PER_SEGMENT * segs) / len(rec) + \
        BYTES_PER_PACKET * N
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9
    add_rates = atomic_peak()
    atom = measured_atomics()
    if atom:
        req_peaks = {p: add_rates[p] * atom["requests_per_add"][p] for p in ATOMIC_PATTERNS}
        atom_peak = max(req_peaks.values())
        atom_rate = atom["requests_per_pass"] / (mean_ms * 1e-3)
    else:
        req_peaks, atom_peak, atom_rate = None, None, None

    out = {
        "metric": "packet-interactions/sec",
        "value": inter / wall,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "shells": w.model.n_shells, "lines": w.model.n_lines,
                   "packets_per_iteration": N, "iterations": args.steps,
                   "T_inner_start": w.T_inner, "line_mode": "scatter",
                   "jblue": not args.no_jblue},
        "packets_per_s": N * args.steps / wall,
        "segments_per_s": segs / wall,
        "line_passes_per_s": passes / wall,
        "transport_ms": kern_ms,
        "T_inner": [t for _, _, t, _ in rec],
        "escape_fraction": [f for _, _, _, f in rec],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "traffic_unit": "HBM bytes per transport pass",
                     "kernel": "transport pass: transport_kernel, order kernels and the "
                               "group kernel of the handed-off histories",
                     "bytes_per_launch": bytes_per_launch,
                     "bytes_model": "16 B per line passed + 24 B per segment + 96 B per packet",
                     "valu": valu_entry(mean_ms),
                     "atomic": {"achieved": atom_rate, "peak": atom_peak,
                                "unit": "L2 atomic requests/s",
                                "frac": atom_rate / atom_peak if atom_rate else None,
                                "requests_per_launch": atom["requests_per_pass"] if atom else None,
                                "peak_by_pattern": req_peaks,
                                "fp64_adds_per_s_by_pattern": add_rates,
                                "source": "TCC_ATOMIC per pass and per calibration add from "
                                          "the committed counter summary (null when the "
                                          "kernel source has changed since); add rates of "
                                          "the two tally patterns measured in this run"}},
        "cpu_baseline": None,
    }
    out["pcie_inclusive"] = host_boundary(ctx, w, flags, N, inter, wall, args.steps)
    out["critical_path"] = None
    if not args.no_critical_path:
        out["critical_path"] = critical_path(ctx, w, flags, args.steps - 1, rec[-1][2],
                                             kern_ms[-1])
        print(f"# critical path: {json.dumps(out['critical_path'])}", file=sys.stderr,
              flush=True)
    if not args.no_batched:
        model.free()
        out["batched"] = batched_measure(args.models, 3, 1, not args.no_jblue, log=True)
        print(f"# batched: {out['batched']['batched']['models_per_s']:.2f} models/s, plain "
              f"{out['batched']['plain']['models_per_s']:.2f}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        schedule = [(i, t) for i, (_, _, t, _) in enumerate(rec)]
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample, args.cpu_procs, schedule)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
